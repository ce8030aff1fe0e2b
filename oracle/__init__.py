"""The oracle: a plain, slow, FP64 CPU reference for the Wilson / Wilson-clover
fermion matrix of eq. (1) (Sec. 3) of the Bridge++ 2.0 paper
(arXiv:2111.04457), its even-odd Schur form, textbook Krylov solvers and the
pseudofermion force.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library: it loads
its own C file (lqoracle.c, built with gcc) and composes it with numpy here.

Array conventions (complex128, C-contiguous):
  U[t, z, y, x, mu, a, b], psi[t, z, y, x, spin, colour], dims = (Lx, Ly, Lz, Lt).
  Parity vectors are [V/2, 4, 3] in checkerboard order cb = lex // 2, where
  lex = x + Lx*(y + Ly*(z + Lz*t)) and parity = (x + y + z + t) mod 2.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.ensure_built()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L = ctypes.c_long
        lib.lqo_gamma.argtypes = [I, P]
        lib.lqo_gamma.restype = I
        lib.lqo_num_threads.restype = I
        lib.lqo_set_num_threads.argtypes = [I]
        lib.lqo_hop.argtypes = [P, P, P, P, P, I]
        lib.lqo_dirac.argtypes = [P, P, P, D, P, P, P, I]
        lib.lqo_dirac_sites.argtypes = [P, P, P, D, P, P, L, P, P, I]
        lib.lqo_hop_sites.argtypes = [P, P, P, P, L, P, P, I]
        lib.lqo_clover.argtypes = [P, P, D, D, I, P]
        lib.lqo_clover_sites.argtypes = [P, P, D, D, I, L, P, P]
        lib.lqo_site_apply.argtypes = [L, P, P, P]
        lib.lqo_site_invert.argtypes = [L, P, P]
        lib.lqo_site_invert.restype = L
        lib.lqo_hop_link_derivative.argtypes = [P, P, P, P, D, P]
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _dims(dims) -> np.ndarray:
    d = np.asarray([int(v) for v in dims], dtype=np.int32)
    assert d.shape == (4,) and np.all(d >= 2) and np.all(d % 2 == 0), "dims must be 4 even sizes >= 2"
    return d


def _bc(bc) -> np.ndarray:
    if bc is None:
        bc = (1, 1, 1, 1)
    out = np.zeros(4, dtype=np.complex128)
    for i, v in enumerate(bc):
        out[i] = complex(*v) if isinstance(v, (tuple, list)) else complex(v)
    return out


def num_threads() -> int:
    return int(_lib().lqo_num_threads())


def set_num_threads(n: int) -> None:
    _lib().lqo_set_num_threads(int(n))


def gamma(mu: int) -> np.ndarray:
    """gamma_{mu+1} for mu = 0..3 (x, y, z, t) or gamma_5 for mu = 4."""
    out = np.zeros((4, 4), dtype=np.complex128)
    if _lib().lqo_gamma(int(mu), _ptr(out)) != 0:
        raise ValueError("mu must be 0..4")
    return out


def volume(dims) -> int:
    return int(np.prod([int(d) for d in dims]))


# ---------------------------------------------------------------- operators


def hop(dims, U, bc, psi, dagger=False) -> np.ndarray:
    """H psi (dagger=False) or H^dag psi: the hopping sum of eq. (1) without -kappa."""
    d = _dims(dims)
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    _lib().lqo_hop(_ptr(d), _ptr(U), _ptr(_bc(bc)), _ptr(psi), _ptr(out), int(bool(dagger)))
    return out


def dirac(dims, U, bc, kappa, psi, F=None, dagger=False) -> np.ndarray:
    """D psi of eq. (1) (or D^dag psi), with clover term F[V,12,12] or F = 0."""
    d = _dims(dims)
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    Fp = None if F is None else _c128(F)
    _lib().lqo_dirac(_ptr(d), _ptr(U), _ptr(_bc(bc)), float(kappa), None if Fp is None else _ptr(Fp),
                     _ptr(psi), _ptr(out), int(bool(dagger)))
    return out


def dirac_sites(dims, U, bc, kappa, psi, sites, F=None, dagger=False) -> np.ndarray:
    """(D psi)(x) at the lexicographic sites listed; returns [n, 4, 3]."""
    d = _dims(dims)
    U = _c128(U)
    psi = _c128(psi)
    s = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(s), 4, 3), dtype=np.complex128)
    Fp = None if F is None else _c128(F)
    _lib().lqo_dirac_sites(_ptr(d), _ptr(U), _ptr(_bc(bc)), float(kappa), None if Fp is None else _ptr(Fp),
                           _ptr(psi), len(s), _ptr(s), _ptr(out), int(bool(dagger)))
    return out


def hop_sites(dims, U, bc, psi, sites, dagger=False) -> np.ndarray:
    d = _dims(dims)
    U = _c128(U)
    psi = _c128(psi)
    s = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(s), 4, 3), dtype=np.complex128)
    _lib().lqo_hop_sites(_ptr(d), _ptr(U), _ptr(_bc(bc)), _ptr(psi), len(s), _ptr(s), _ptr(out),
                         int(bool(dagger)))
    return out


def clover(dims, U, csw, kappa, traceless=True) -> np.ndarray:
    """F(x) as [V, 12, 12] (index spin*3 + colour)."""
    d = _dims(dims)
    U = _c128(U)
    V = volume(dims)
    F = np.empty((V, 12, 12), dtype=np.complex128)
    _lib().lqo_clover(_ptr(d), _ptr(U), float(csw), float(kappa), int(bool(traceless)), _ptr(F))
    return F


def clover_sites(dims, U, csw, kappa, sites, traceless=True) -> np.ndarray:
    d = _dims(dims)
    U = _c128(U)
    s = np.ascontiguousarray(sites, dtype=np.int64)
    F = np.empty((len(s), 12, 12), dtype=np.complex128)
    _lib().lqo_clover_sites(_ptr(d), _ptr(U), float(csw), float(kappa), int(bool(traceless)), len(s),
                            _ptr(s), _ptr(F))
    return F


def site_apply(M, psi) -> np.ndarray:
    """out[x] = M[x] psi[x] for 12x12 site matrices."""
    M = _c128(M)
    psi = _c128(psi)
    n = M.shape[0]
    assert psi.size == n * 12
    out = np.empty_like(psi)
    _lib().lqo_site_apply(n, _ptr(M), _ptr(psi), _ptr(out))
    return out


def site_invert(M):
    """(Minv, n_singular): per-site 12x12 inverse by Gauss-Jordan with partial pivoting."""
    M = _c128(M)
    n = M.shape[0]
    out = np.empty_like(M)
    nsing = _lib().lqo_site_invert(n, _ptr(M), _ptr(out))
    return out, int(nsing)


def hop_link_derivative(dims, bc, a, b, coef=1.0, out=None) -> np.ndarray:
    """M[t,z,y,x,mu,3,3] with d Re[a^dag H b] = sum Re tr(M dU); accumulated into out."""
    d = _dims(dims)
    a = _c128(a)
    b = _c128(b)
    if out is None:
        out = np.zeros(tuple(int(v) for v in dims[::-1]) + (4, 3, 3), dtype=np.complex128)
    assert out.dtype == np.complex128 and out.flags.c_contiguous
    _lib().lqo_hop_link_derivative(_ptr(d), _ptr(_bc(bc)), _ptr(a), _ptr(b), float(coef), _ptr(out))
    return out


# --------------------------------------------------------------- even-odd


def parity_of_sites(dims) -> np.ndarray:
    """parity (x+y+z+t) mod 2 of every lexicographic site."""
    lx, ly, lz, lt = (int(v) for v in dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return ((x + y + z + t) % 2).reshape(-1)


def parity_sites(dims, p) -> np.ndarray:
    """Lexicographic indices of the sites of parity p, in checkerboard order:
    the k-th entry is the site with lex // 2 == k."""
    par = parity_of_sites(dims)
    idx = np.nonzero(par == p)[0]
    assert np.array_equal(idx // 2, np.arange(len(idx)))
    return idx


def to_parity(dims, psi, p) -> np.ndarray:
    """Full field [.., 4, 3] -> [V/2, 4, 3] restricted to parity p."""
    V = volume(dims)
    return np.ascontiguousarray(psi.reshape(V, 4, 3)[parity_sites(dims, p)])


def from_parity(dims, half, p, out=None) -> np.ndarray:
    """[V/2, 4, 3] on parity p -> full field (other parity zero unless out given)."""
    V = volume(dims)
    if out is None:
        out = np.zeros((V, 4, 3), dtype=np.complex128)
    else:
        out = out.reshape(V, 4, 3)
    out[parity_sites(dims, p)] = half.reshape(-1, 4, 3)
    return out.reshape(tuple(int(v) for v in dims[::-1]) + (4, 3))


def twist_term(V, twist) -> np.ndarray:
    """i tau gamma_5 (x) 1_colour at every site, [V, 12, 12]: the twisted-mass
    term of the Wilson operator D = 1 - kappa H + i tau gamma_5 (tau = 2 kappa mu
    for a twisted mass mu in the normalisation of eq. (1))."""
    g5 = np.kron(np.diag([1.0, 1.0, -1.0, -1.0]), np.eye(3)).astype(np.complex128)
    return np.broadcast_to(1j * float(twist) * g5, (V, 12, 12)).copy()


class Operator:
    """The fermion matrix D = A - kappa H with A = 1 + F on one gauge field,
    and its even-odd blocks D = [[A_ee, -kappa H_eo], [-kappa H_oe, A_oo]].
    With twist != 0, F also holds the twisted-mass term i twist gamma_5
    (A is then not Hermitian)."""

    def __init__(self, dims, U, kappa, csw=0.0, bc=None, traceless=True, twist=0.0):
        self.dims = tuple(int(v) for v in dims)
        self.V = volume(dims)
        self.U = _c128(U)
        self.kappa = float(kappa)
        self.csw = float(csw)
        self.twist = float(twist)
        self.bc = _bc(bc)
        self.shape = tuple(self.dims[::-1]) + (4, 3)
        F = clover(self.dims, self.U, self.csw, self.kappa, traceless) if self.csw != 0.0 else None
        if self.twist != 0.0:
            F = twist_term(self.V, self.twist) if F is None else F + twist_term(self.V, self.twist)
        if F is not None:
            self.F = F
            A = self.F + np.eye(12)[None]
            self.A = A
            self.Ainv, nsing = site_invert(A)
            if nsing:
                raise ZeroDivisionError("%d singular clover blocks" % nsing)
        else:
            self.F = None
            self.A = None
            self.Ainv = None
        self.sites = (parity_sites(self.dims, 0), parity_sites(self.dims, 1))

    # full lattice
    def D(self, psi):
        return dirac(self.dims, self.U, self.bc, self.kappa, psi.reshape(self.shape), self.F, False)

    def Ddag(self, psi):
        return dirac(self.dims, self.U, self.bc, self.kappa, psi.reshape(self.shape), self.F, True)

    def DdagD(self, psi):
        return self.Ddag(self.D(psi))

    def H(self, psi, dagger=False):
        return hop(self.dims, self.U, self.bc, psi.reshape(self.shape), dagger)

    # parity blocks (vectors [V/2, 4, 3])
    def hop_to(self, p_out, v_in, dagger=False):
        """H_{p_out, 1-p_out} v (or the block of H^dag): output on parity p_out."""
        full = from_parity(self.dims, v_in, 1 - p_out)
        return to_parity(self.dims, hop(self.dims, self.U, self.bc, full, dagger), p_out)

    def clover_apply(self, p, v, inverse=False, dagger=False):
        if self.A is None:
            return v.copy()
        M = (self.Ainv if inverse else self.A)[self.sites[p]]
        if dagger:
            M = np.ascontiguousarray(np.conj(np.swapaxes(M, 1, 2)))
        return site_apply(M, v).reshape(v.shape)

    def schur(self, xe):
        """M = A_ee - kappa^2 H_eo A_oo^-1 H_oe."""
        t = self.clover_apply(1, self.hop_to(1, xe), inverse=True)
        return self.clover_apply(0, xe) - self.kappa ** 2 * self.hop_to(0, t)

    def schur_dag(self, xe):
        """M^dag = A_ee^dag - kappa^2 (H_oe)^dag (A_oo^-1)^dag (H_eo)^dag."""
        t = self.clover_apply(1, self.hop_to(1, xe, dagger=True), inverse=True, dagger=True)
        return self.clover_apply(0, xe, dagger=True) - self.kappa ** 2 * self.hop_to(0, t, dagger=True)

    def schur_normal(self, xe):
        return self.schur_dag(self.schur(xe))

    def prepare(self, b):
        """b_hat_e = b_e + kappa H_eo A_oo^-1 b_o."""
        be = to_parity(self.dims, b, 0)
        bo = to_parity(self.dims, b, 1)
        return be + self.kappa * self.hop_to(0, self.clover_apply(1, bo, inverse=True))

    def reconstruct(self, b, xe):
        """x_o = A_oo^-1 (b_o + kappa H_oe x_e); returns the full solution."""
        bo = to_parity(self.dims, b, 1)
        xo = self.clover_apply(1, bo + self.kappa * self.hop_to(1, xe), inverse=True)
        x = from_parity(self.dims, xe, 0)
        return from_parity(self.dims, xo, 1, out=x)


# ---------------------------------------------------------------- solvers


def _dot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def _nrm2(a):
    return float(np.vdot(a.reshape(-1), a.reshape(-1)).real)


def cg(apply_A, rhs, tol, max_iter=100000, x0=None):
    """Hestenes-Stiefel conjugate gradients for a Hermitian positive-definite
    A; stops when |r| <= tol |rhs| on the recursive residual, then recomputes
    the true residual and continues if it is not met.  Returns (x, iters)."""
    x = np.zeros_like(rhs) if x0 is None else x0.copy()
    bn = np.sqrt(_nrm2(rhs))
    if bn == 0.0:
        return np.zeros_like(rhs), 0
    r = rhs - apply_A(x) if x0 is not None else rhs.copy()
    p = r.copy()
    rr = _nrm2(r)
    it = 0
    while it < max_iter:
        if np.sqrt(rr) <= tol * bn:
            r = rhs - apply_A(x)
            rr = _nrm2(r)
            if np.sqrt(rr) <= tol * bn:
                break
            p = r.copy()
        q = apply_A(p)
        alpha = rr / _dot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rr_new = _nrm2(r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def bicgstab(apply_A, rhs, tol, max_iter=100000, x0=None):
    """BiCGStab of van der Vorst (1992) with shadow residual r_hat = r_0;
    restarts from the current iterate when rho or omega vanish.  Stops on
    the recursive residual, then confirms on the true residual.  Returns
    (x, iters)."""
    x = np.zeros_like(rhs) if x0 is None else x0.copy()
    bn = np.sqrt(_nrm2(rhs))
    if bn == 0.0:
        return np.zeros_like(rhs), 0
    it = 0
    while it < max_iter:
        r = rhs - apply_A(x)
        if np.sqrt(_nrm2(r)) <= tol * bn:
            break
        rhat = r.copy()
        rho = alpha = omega = 1.0
        v = np.zeros_like(r)
        p = np.zeros_like(r)
        restart = False
        while it < max_iter:
            rho_new = _dot(rhat, r)
            if abs(rho_new) < 1e-30 * bn * bn:
                restart = True
                break
            beta = (rho_new / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
            v = apply_A(p)
            alpha = rho_new / _dot(rhat, v)
            s = r - alpha * v
            t = apply_A(s)
            tt = _nrm2(t)
            omega = _dot(t, s) / tt if tt > 0 else 0.0
            x = x + alpha * p + omega * s
            r = s - omega * t
            rho = rho_new
            it += 1
            if np.sqrt(_nrm2(r)) <= tol * bn:
                break
            if abs(omega) < 1e-30:
                restart = True
                break
        if not restart and np.sqrt(_nrm2(rhs - apply_A(x))) <= tol * bn:
            break
    return x, it


def solve_eo(op: Operator, b, tol=1e-12, method="bicgstab", max_iter=100000):
    """x = D^-1 b by the even-odd Schur complement.  Returns (x, iters)."""
    bh = op.prepare(b)
    if method == "bicgstab":
        xe, it = bicgstab(op.schur, bh, tol * 0.5, max_iter)
    else:
        xe, it = cg(op.schur_normal, op.schur_dag(bh), tol * 0.1, max_iter)
    return op.reconstruct(b, xe), it


def true_residual(op: Operator, x, b) -> float:
    """|b - D x| / |b| in FP64 (2-norm over all sites and components)."""
    bn = np.linalg.norm(b.reshape(-1))
    if bn == 0.0:
        return 0.0
    return float(np.linalg.norm((b - op.D(x)).reshape(-1)) / bn)


# ------------------------------------------------------------------ force


def traceless_antihermitian(m) -> np.ndarray:
    """TA(m) = (m - m^dag)/2 - tr(m - m^dag)/6 on the last two axes."""
    a = 0.5 * (m - np.conj(np.swapaxes(m, -1, -2)))
    tr = np.trace(a, axis1=-2, axis2=-1) / 3.0
    return a - tr[..., None, None] * np.eye(3)


def pf_action_eo(op: Operator, phi_e, tol=1e-13):
    """S = phi_e^dag (M^dag M)^-1 phi_e for the Wilson even-odd operator
    M = 1 - kappa^2 H_eo H_oe.  Returns (S, X) with X = (M^dag M)^-1 phi_e."""
    X, _ = cg(op.schur_normal, phi_e, tol)
    return float(_dot(phi_e, X).real), X


def pf_force_eo(op: Operator, phi_e, tol=1e-13):
    """Pseudofermion force of S = phi_e^dag (M^dag M)^-1 phi_e (Wilson,
    even-odd).  With X = (M^dag M)^-1 phi_e, Y = M X, Z = H_oe X,
    W = (H_eo)^dag Y one has dS = 2 kappa^2 Re[Y^dag dH_eo Z + W^dag dH_oe X].
    Returns (S, Mraw, G): Mraw[.., mu, 3, 3] with dS = sum Re tr(Mraw dU) and
    the su(3) force G = -TA(U Mraw)."""
    assert op.F is None, "the even-odd force is for the Wilson operator"
    S, X = pf_action_eo(op, phi_e, tol)
    Y = op.schur(X)
    Z = op.hop_to(1, X)
    W = op.hop_to(1, Y, dagger=True)
    d = op.dims
    k2 = op.kappa ** 2
    Mraw = hop_link_derivative(d, op.bc, from_parity(d, Y, 0), from_parity(d, Z, 1), 2.0 * k2)
    hop_link_derivative(d, op.bc, from_parity(d, W, 1), from_parity(d, X, 0), 2.0 * k2, out=Mraw)
    G = -traceless_antihermitian(op.U @ Mraw)
    return S, Mraw, G


def pf_force_full(op: Operator, phi, tol=1e-13):
    """S = phi^dag (D^dag D)^-1 phi (Wilson, full lattice): with
    X = (D^dag D)^-1 phi and Y = D X, dS = 2 kappa Re[Y^dag dH X].
    Returns (S, Mraw, G)."""
    assert op.F is None
    X, _ = cg(op.DdagD, phi.reshape(op.shape), tol)
    S = float(_dot(phi, X).real)
    Y = op.D(X)
    Mraw = hop_link_derivative(op.dims, op.bc, Y, X, 2.0 * op.kappa)
    G = -traceless_antihermitian(op.U @ Mraw)
    return S, Mraw, G
