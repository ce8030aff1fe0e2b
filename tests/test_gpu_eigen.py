"""The lowest eigenpairs of M^dag M (lq_eigs: thick-restart Lanczos with
full reorthogonalisation on the GPU, plain or on a Chebyshev filter)
against the oracle: the eigenvalues of the dense even-odd normal matrix
built entry by entry from eq. (1) (oracle/dense.py) on 4^4, the
free-field closed form of the lowest one, and the oracle's own M^dag M
applied to the returned vectors.

Tolerances: the Ritz values of converged pairs are within |r|^2 / gap of
the eigenvalues; with residuals below 1e-9 relative, 1e-10 relative is
asserted on the eigenvalues and 1e-8 on the oracle residual of the vectors.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import gauge_exp, gauge_unit, gaussian_parity_spinor
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

BC = (1.0, np.exp(0.3j), 1.0, -1.0)


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


def _dense_normal_eigs(dims, U, kappa, csw, bc):
    from oracle.dense import dense_dirac, parity_index
    D = dense_dirac(dims, U, kappa, csw, bc)
    ie, io = parity_index(dims, 0), parity_index(dims, 1)
    M = D[np.ix_(ie, ie)] - D[np.ix_(ie, io)] @ np.linalg.solve(D[np.ix_(io, io)], D[np.ix_(io, ie)])
    return np.linalg.eigvalsh(M.conj().T @ M)


# (m, restarts allowed, Chebyshev degree): one long cycle; short cycles
# with thick restarts; the filter with its interval picked automatically
CASES = [(200, 0, 0), (20, 200, 0), (24, 50, 12)]


@pytest.mark.parametrize("csw", [0.0, 1.7])
@pytest.mark.parametrize("m,restarts,degree", CASES)
def test_lowest_eigenvalues_match_dense_oracle(lq, csw, m, restarts, degree):
    dims = (4, 4, 4, 4)
    kappa = 0.12
    U = gauge_exp(dims, 0.4, 7101)
    announce("eigs 4^4 csw=%g m=%d restarts<=%d degree=%d" % (csw, m, restarts, degree))
    want = _dense_normal_eigs(dims, U, kappa, csw, BC)
    op = lq.Operator(dims, kappa, csw, BC)
    op.set_gauge(to_dev(U))
    nev = 6
    ev, res, X, st = op.eigs(nev, m, v0=to_dev(gaussian_parity_spinor(dims, 7102)), tol=1e-9, vectors=True,
                             max_restarts=restarts, cheb_degree=degree)
    announce("  evals %s\n  dense %s\n  resid %s\n  %s" % (np.array(ev), want[:nev], np.array(res), st))
    assert st["nconv"] == nev
    assert np.allclose(ev, want[:nev], rtol=1e-10, atol=0)
    if restarts == 0:
        assert st["restarts"] == 0
    if degree:
        # the automatic interval brackets the spectrum above the wanted values
        # (lo is a Ritz value of a plain cycle, not below the (nev+1)-th
        # eigenvalue by interlacing; hi estimates the largest eigenvalue)
        assert want[nev] <= st["cheb_lo"] < st["cheb_hi"] and st["cheb_hi"] >= 0.9 * want[-1]
    # the vectors: orthonormal, and eigenvectors of the oracle's M^dag M
    Xh = to_host(X).reshape(nev, -1)
    gram = Xh.conj() @ Xh.T
    assert np.abs(gram - np.eye(nev)).max() < 1e-10
    ref = oracle.Operator(dims, U, kappa, csw, BC)
    for k in range(nev):
        xk = to_host(X[k])
        r = ref.schur_normal(xk) - ev[k] * xk
        assert np.linalg.norm(r) / (ev[k] * np.linalg.norm(xk)) < 1e-8
    op.close()


def test_free_field_lowest_eigenvalue(lq):
    """At U = 1 the even-odd operator is diagonal in momentum: its
    eigenvalues are 1 - kappa^2 w^2 with w the eigenvalues of
    2 sum cos p - 2i sum gamma_mu sin p, so the smallest eigenvalue of
    M^dag M is the smallest |1 - kappa^2 w^2|^2 over the momenta."""
    dims = (4, 4, 4, 8)
    theta = (0.0, 0.0, 0.0, np.pi)
    kappa = 0.115
    g = [oracle.gamma(mu) for mu in range(4)]
    best = np.inf
    for n0 in range(dims[0]):
        for n1 in range(dims[1]):
            for n2 in range(dims[2]):
                for n3 in range(dims[3]):
                    p = [(2 * np.pi * n + th) / L for n, th, L in zip((n0, n1, n2, n3), theta, dims)]
                    Hp = 2 * sum(np.cos(p)) * np.eye(4) - 2j * sum(g[m] * np.sin(p[m]) for m in range(4))
                    w = np.linalg.eigvals(Hp)
                    best = min(best, float(np.min(np.abs(1 - kappa ** 2 * w ** 2) ** 2)))
    op = lq.Operator(dims, kappa, 0.0, (1, 1, 1, -1))
    op.set_gauge(to_dev(gauge_unit(dims)))
    ev, res, _, st = op.eigs(1, 60, v0=to_dev(gaussian_parity_spinor(dims, 7201)), tol=1e-10, cheb_degree=0)
    announce("  free field: lowest %.15e, closed form %.15e, resid %.1e" % (ev[0], best, res[0]))
    assert st["nconv"] == 1 and abs(ev[0] - best) < 1e-10 * best
    op.close()


@pytest.mark.parametrize("degree", [0, 16])
def test_eigs_8x8x8x8_properties(lq, degree):
    """Larger lattice, short cycles with thick restarts, plain and filtered:
    converged residuals, ascending values, the same eigenvalues both ways,
    and the smallest below the Rayleigh quotient of random vectors."""
    import torch
    dims = (8, 8, 8, 8)
    U = gauge_exp(dims, 0.3, 7301)
    op = lq.Operator(dims, 0.125, 1.0, (1, 1, 1, -1))
    op.set_gauge(to_dev(U))
    ev, res, X, st = op.eigs(8, 40, v0=to_dev(gaussian_parity_spinor(dims, 7302)), tol=1e-8, vectors=True,
                             cheb_degree=degree)
    announce("  8^4 degree %d evals %s resid %s %s" % (degree, np.array(ev), np.array(res), st))
    assert st["nconv"] == 8 and all(ev[i] <= ev[i + 1] for i in range(7))
    assert all(r <= 1e-8 * e for r, e in zip(res, ev))
    for seed in (7303, 7304):
        v = to_dev(gaussian_parity_spinor(dims, seed))
        Av = op.apply("schur_normal", v, "f64")
        rq = float(torch.vdot(v.reshape(-1), Av.reshape(-1)).real / torch.vdot(v.reshape(-1), v.reshape(-1)).real)
        assert ev[0] < rq
    # the other variant agrees on the eigenvalues; it reuses the workspace
    # the first call left with the operator
    kib = op.get_option("work_kib")
    ev2, _, _, st2 = op.eigs(8, 40, v0=to_dev(gaussian_parity_spinor(dims, 7305)), tol=1e-8,
                             cheb_degree=16 - degree)
    assert st2["nconv"] == 8 and np.allclose(ev, ev2, rtol=1e-12, atol=0)
    assert op.get_option("work_kib") == kib > 0
    # a repeated call on the kept workspace gives the same bits
    ev3, res3, X3, _ = op.eigs(8, 40, v0=to_dev(gaussian_parity_spinor(dims, 7302)), tol=1e-8, vectors=True,
                               cheb_degree=degree)
    assert list(ev3) == list(ev) and list(res3) == list(res) and np.array_equal(to_host(X3), to_host(X))
    op.close()


def test_eigs_argument_checks(lq):
    import ctypes
    from paper_2111_04457_amd import _lib
    lib = _lib.load()
    op = lq.Operator((4, 4, 4, 4), 0.12, 0.0, (1, 1, 1, -1))
    ev = (ctypes.c_double * 16)()
    dummy = ctypes.c_void_p(16)  # never dereferenced: the checks fail first

    def params(**kw):
        p = _lib.EigParams()
        lib.lq_eig_params_default(ctypes.byref(p))
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    for bad in (dict(nev=4, m=4), dict(nev=0), dict(m=1025), dict(tol=0.0), dict(max_restarts=-1),
                dict(cheb_degree=-1), dict(cheb_degree=10001), dict(cheb_lo=-1.0), dict(cheb_lo=2.0, cheb_hi=1.0),
                dict(cheb_hi=float("inf"))):
        p = params(**bad)
        assert lib.lq_eigs(op.handle, ctypes.byref(p), dummy, ev, None, None, None, None) == -1, bad
    assert lib.lq_eigs(op.handle, None, dummy, ev, None, None, None, None) == -1
    p = params()
    assert lib.lq_eigs(op.handle, ctypes.byref(p), dummy, ev, None, None, None, None) == -2  # no gauge field
    op.set_gauge(to_dev(gauge_unit((4, 4, 4, 4))))
    # a degree whose T_d would overflow on the interval
    p = params(cheb_degree=5000, cheb_lo=1.0, cheb_hi=2.0)
    v0 = to_dev(gaussian_parity_spinor((4, 4, 4, 4), 7401))
    assert lib.lq_eigs(op.handle, ctypes.byref(p), ctypes.c_void_p(v0.data_ptr()), ev, None, None, None,
                       None) == -1
    op.close()


def test_deflated_guess_matches_oracle(lq):
    """lq_deflated_guess against the oracle: eigenvectors of the dense
    M^dag M (oracle/dense.py) as input, the guess composed from the oracle's
    prepare, M^dag and reconstruct; the even residual of the guess has no
    component along M^dag of the eigenvectors' span."""
    from oracle.dense import dense_dirac, parity_index
    from lattice_inputs import gaussian_spinor
    dims = (4, 4, 4, 4)
    kappa, csw = 0.12, 1.7
    U = gauge_exp(dims, 0.4, 7501)
    D = dense_dirac(dims, U, kappa, csw, BC)
    ie, io = parity_index(dims, 0), parity_index(dims, 1)
    M = D[np.ix_(ie, ie)] - D[np.ix_(ie, io)] @ np.linalg.solve(D[np.ix_(io, io)], D[np.ix_(io, ie)])
    w, Z = np.linalg.eigh(M.conj().T @ M)
    nvec = 6
    Vh = np.ascontiguousarray(Z[:, :nvec].T).reshape((nvec,) + (dims[0] * dims[1] * dims[2] * dims[3] // 2, 4, 3))
    ref = oracle.Operator(dims, U, kappa, csw, BC)
    for k in range(nvec):  # the dense ordering is the parity fields' ordering
        assert np.linalg.norm(ref.schur_normal(Vh[k]) - w[k] * Vh[k]) < 1e-10 * w[k]
    b = gaussian_spinor(dims, 7502)
    bh = ref.prepare(b)
    y = ref.schur_dag(bh)
    xe = sum(np.vdot(Vh[k], y) / w[k] * Vh[k] for k in range(nvec))
    want = ref.reconstruct(b, xe)
    op = lq.Operator(dims, kappa, csw, BC)
    op.set_gauge(to_dev(U))
    x0 = to_host(op.deflated_guess(to_dev(b), list(w[:nvec]), to_dev(Vh)))
    err = np.linalg.norm(x0.reshape(-1) - want.reshape(-1)) / np.linalg.norm(want)
    announce("  deflated guess vs oracle %.2e" % err)
    assert err < 1e-12
    from oracle import to_parity
    r = bh - ref.schur(to_parity(dims, x0, 0))
    g = ref.schur_dag(r)
    proj = max(abs(np.vdot(Vh[k], g)) for k in range(nvec))
    assert proj < 1e-10 * max(abs(np.vdot(Vh[k], y)) for k in range(nvec))
    # the odd rows of D x0 = b hold
    assert np.linalg.norm(to_parity(dims, ref.D(x0) - b, 1)) < 1e-12 * np.linalg.norm(b)
    op.close()


def test_deflated_solve_8x8x8x8(lq):
    """Eigenvectors from lq_eigs deflate the start of a mixed solve: both
    starts reach the tolerance and the same solution."""
    from lattice_inputs import gaussian_spinor
    dims = (8, 8, 8, 8)
    op = lq.Operator(dims, 0.125, 1.0, (1, 1, 1, -1))
    op.set_gauge(to_dev(gauge_exp(dims, 0.3, 7601)))
    ev, res, X, st = op.eigs(16, 64, v0=to_dev(gaussian_parity_spinor(dims, 7602)), tol=1e-10, vectors=True)
    assert st["nconv"] == 16
    b = to_dev(gaussian_spinor(dims, 7603))
    prm = lq.SolverParams(solver="bicgstab", tol=1e-10, inner="f32")
    x_plain, s_plain = op.solve(b, "D", prm)
    x0 = op.deflated_guess(b, ev, X)
    x_defl, s_defl = op.solve(b, "D", prm, x0=x0)
    announce("  inner iterations: zero start %d, deflated start %d" % (s_plain[0].nconv, s_defl[0].nconv))
    assert s_plain[0].converged and s_defl[0].converged
    assert rel_err(to_host(x_defl), to_host(x_plain)) < 1e-8


def test_deflated_guess_argument_checks(lq):
    import ctypes
    from paper_2111_04457_amd import _lib
    lib = _lib.load()
    op = lq.Operator((4, 4, 4, 4), 0.12, 0.0, (1, 1, 1, -1))
    dummy = ctypes.c_void_p(16)  # never dereferenced: the checks fail first
    ev = (ctypes.c_double * 2)(0.5, 0.7)
    bad = (ctypes.c_double * 2)(0.5, -0.7)
    assert lib.lq_deflated_guess(op.handle, 0, ev, dummy, dummy, dummy, None) == -1
    assert lib.lq_deflated_guess(op.handle, 2, bad, dummy, dummy, dummy, None) == -1
    assert lib.lq_deflated_guess(op.handle, 2, ev, None, dummy, dummy, None) == -1
    assert lib.lq_deflated_guess(op.handle, 2, ev, dummy, dummy, dummy, None) == -2  # no gauge field
    op.close()


def test_eigs_16x16x16x32_workload_against_oracle(lq):
    """The timed configuration (16^3x32 clover workload, 8 lowest modes,
    64 basis vectors per cycle, degree-8 filter with the automatic
    interval): the returned vectors are checked with the oracle's own
    M^dag M, pair by pair, and for orthonormality."""
    from lattice_inputs import ANTIPERIODIC_T, WORKLOADS, workload_gauge
    name = "clover_16x16x16x32"
    w = WORKLOADS[name]
    dims = w["dims"]
    U = workload_gauge(name)
    op = lq.Operator(dims, w["kappa"], w["csw"], ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    ev, res, X, st = op.eigs(8, 64, v0=to_dev(gaussian_parity_spinor(dims, 2008)), tol=1e-8, vectors=True)
    announce("  %s: %s, lowest %.6e, largest resid %.1e" % (name, st, ev[0], max(res)))
    assert st["nconv"] == 8
    # the pairs are from the wanted end: every eigenvalue below the filter's
    # lower edge (which lies above the 9th eigenvalue)
    assert max(ev) <= st["cheb_lo"] < st["cheb_hi"]
    Xh = to_host(X).reshape(8, -1)
    assert np.abs(Xh.conj() @ Xh.T - np.eye(8)).max() < 1e-10
    ref = oracle.Operator(dims, U, w["kappa"], w["csw"], ANTIPERIODIC_T)
    for k in (0, 3, 7):
        xk = to_host(X[k])
        Ax = ref.schur_normal(xk)
        lam = float(np.vdot(xk.reshape(-1), Ax.reshape(-1)).real)
        r = np.linalg.norm(Ax - ev[k] * xk)
        announce("    pair %d: GPU %.15e oracle Rayleigh %.15e, oracle residual %.1e" % (k, ev[k], lam, r / ev[k]))
        assert abs(lam - ev[k]) < 1e-12 * ev[k]
        assert r < 2e-8 * ev[k]
    op.close()
