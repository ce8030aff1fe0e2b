"""Pseudofermion action and force of the Wilson-clover operator written as
the gradient of the action (the molecular-dynamics force of the gauge-field
generation of Sec. 2, for the fermion matrix of eq. (1)).

TEST INFRASTRUCTURE ONLY.  The action

    even-odd:      S = phi_e^dag (M^dag M)^-1 phi_e,  M = A_ee - kappa^2 H_eo A_oo^-1 H_oe
    full lattice:  S = phi^dag (D^dag D)^-1 phi

is evaluated from a dense D built with torch CPU operations in FP64 straight
from eq. (1): hopping blocks -kappa kron(1 -+ gamma_mu, U) with the boundary
phases, and the clover term -c_sw kappa sum_{mu<nu} gamma_mu gamma_nu (x)
Fhat_{mu nu} with Fhat = (Q - Q^dag)/8 from the four counter-clockwise
leaves.  torch autograd then gives dS/dU, so the force is the definition of
the derivative itself, with no hand-derived formula.  Dense N x N matrices
(N = 12 V): tiny lattices only.

pf_force_clover_mf reaches larger lattices: X comes from the conjugate-
gradient solve of the C oracle, and only the step that follows from the
definition is left to autograd: with Y = M X (M the matrix of the action),
dS = -X^dag d(M^dag M) X = -2 Re[Y^dag dM X], so the gradient is -2 times
that of the bilinear Re[Y^dag M(U) X] with X, Y held fixed, where M(U) X is
evaluated matrix-free (neighbour shifts, per-site 12 x 12 blocks).
"""
from __future__ import annotations

import numpy as np
import torch

from . import Operator, cg, dense as _dense, from_parity, traceless_antihermitian

_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}  # direction mu -> axis of [t, z, y, x]


def _gammas():
    g, _ = _dense.chiral_gammas()
    return [torch.from_numpy(np.asarray(m, dtype=np.complex128)) for m in g]


def _fwd(T, mu):
    """T(x + mu) at site x."""
    return torch.roll(T, shifts=-1, dims=_AXIS[mu])


def _bwd(T, mu):
    """T(x - mu) at site x."""
    return torch.roll(T, shifts=1, dims=_AXIS[mu])


def _h(T):
    return T.conj().transpose(-1, -2)


def _site_blocks(U, dims, kappa, csw, traceless, twist=0.0):
    """Diagonal blocks A(x) = 1 + F(x) (+ i twist gamma_5, the twisted-mass
    term, which does not depend on the links), [Lt, Lz, Ly, Lx, 12, 12]."""
    g = _gammas()
    shape = U.shape[:4]
    A = torch.eye(12, dtype=torch.complex128).expand(*shape, 12, 12).clone()
    if twist != 0.0:
        g5 = torch.from_numpy(np.kron(np.diag([1.0, 1.0, -1.0, -1.0]), np.eye(3)).astype(np.complex128))
        A = A + 1j * float(twist) * g5
    if csw == 0.0:
        return A
    Um = [U[..., mu, :, :] for mu in range(4)]
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a, b = Um[mu], Um[nu]
            # the four counter-clockwise leaves at x
            l1 = a @ _fwd(b, mu) @ _h(_fwd(a, nu)) @ _h(b)
            l2 = b @ _h(_fwd(_bwd(a, mu), nu)) @ _h(_bwd(b, mu)) @ _bwd(a, mu)
            l3 = _h(_bwd(a, mu)) @ _h(_bwd(_bwd(b, mu), nu)) @ _bwd(_bwd(a, mu), nu) @ _bwd(b, nu)
            l4 = _h(_bwd(b, nu)) @ _bwd(a, nu) @ _bwd(_fwd(b, mu), nu) @ _h(a)
            Q = l1 + l2 + l3 + l4
            Fh = (Q - _h(Q)) / 8.0
            if traceless:
                tr = torch.diagonal(Fh, dim1=-2, dim2=-1).sum(-1) / 3.0
                Fh = Fh - tr[..., None, None] * torch.eye(3, dtype=torch.complex128)
            G = g[mu] @ g[nu]
            # kron(G, Fh) with index 3 * spin + colour
            K = torch.einsum("st,...cd->...sctd", G, Fh).reshape(*shape, 12, 12)
            A = A + (-csw * kappa) * K
    return A


def dense_dirac_torch(U, dims, kappa, csw=0.0, bc=(1, 1, 1, 1), traceless=True, twist=0.0):
    """The N x N matrix D = A - kappa H of eq. (1) as a differentiable torch
    tensor (index 12 * lex + 3 * spin + colour); twist != 0 adds
    i twist gamma_5 on every site."""
    dims = tuple(int(v) for v in dims)
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    N = 12 * V
    g = _gammas()
    one = torch.eye(4, dtype=torch.complex128)
    t, z, y, x = torch.meshgrid(torch.arange(lt), torch.arange(lz), torch.arange(ly), torch.arange(lx),
                                indexing="ij")
    coord = [x, y, z, t]
    lex = x + lx * (y + ly * (z + lz * t))
    off = torch.arange(12)
    rows_all, cols_all, vals_all = [], [], []

    def add(rows_site, cols_site, blocks):
        r = (12 * rows_site.reshape(-1, 1, 1) + off.view(1, 12, 1)).expand(-1, 12, 12)
        c = (12 * cols_site.reshape(-1, 1, 1) + off.view(1, 1, 12)).expand(-1, 12, 12)
        rows_all.append(r.reshape(-1))
        cols_all.append(c.reshape(-1))
        vals_all.append(blocks.reshape(-1))

    A = _site_blocks(U, dims, kappa, csw, traceless, twist)
    add(lex, lex, A)
    for mu in range(4):
        L = dims[mu]
        u = U[..., mu, :, :]
        wrap_f = (coord[mu] == L - 1)
        wrap_b = (coord[mu] == 0)
        ph = complex(bc[mu])
        phf = torch.where(wrap_f, torch.tensor(ph, dtype=torch.complex128), torch.tensor(1.0 + 0j, dtype=torch.complex128))
        phb = torch.where(wrap_b, torch.tensor(np.conj(ph), dtype=torch.complex128),
                          torch.tensor(1.0 + 0j, dtype=torch.complex128))
        kf = torch.einsum("st,...cd->...sctd", one - g[mu], u).reshape(*u.shape[:4], 12, 12)
        add(lex, _fwd(lex, mu), -kappa * phf[..., None, None] * kf)
        kb = torch.einsum("st,...cd->...sctd", one + g[mu], _h(_bwd(u, mu))).reshape(*u.shape[:4], 12, 12)
        add(lex, _bwd(lex, mu), -kappa * phb[..., None, None] * kb)
    D = torch.zeros((N, N), dtype=torch.complex128)
    return D.index_put((torch.cat(rows_all), torch.cat(cols_all)), torch.cat(vals_all), accumulate=True)


def _action(U, dims, kappa, csw, bc, traceless, phi, variant, twist=0.0):
    D = dense_dirac_torch(U, dims, kappa, csw, bc, traceless, twist)
    if variant == "eo":
        ie = torch.from_numpy(_dense.parity_index(dims, 0))
        io = torch.from_numpy(_dense.parity_index(dims, 1))
        Dee, Deo = D[ie][:, ie], D[ie][:, io]
        Doe, Doo = D[io][:, ie], D[io][:, io]
        M = Dee - Deo @ torch.linalg.solve(Doo, Doe)
    else:
        M = D
    y = torch.linalg.solve(_h(M), phi)
    return (y.conj() * y).real.sum()


def pf_force_clover(dims, U, kappa, csw, bc, phi, variant="eo", traceless=True, twist=0.0):
    """(S, Mraw, G) for the even-odd ("eo", phi a parity field [V/2, 4, 3] on
    the even sites) or full-lattice ("full", phi [.., 4, 3] over all sites)
    action.  Mraw[t, z, y, x, mu] is the matrix with dS = sum Re tr(Mraw dU);
    G = -TA(U Mraw) is the su(3) force (dS/de along U -> exp(e X) U equals
    sum Re tr(G^dag X))."""
    dims = tuple(int(v) for v in dims)
    Ut = torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128)).clone().requires_grad_(True)
    ph = torch.from_numpy(np.ascontiguousarray(phi, dtype=np.complex128)).reshape(-1)
    S = _action(Ut, dims, float(kappa), float(csw), bc, traceless, ph, variant, twist)
    S.backward()
    # torch returns, for a real function of complex inputs, the gradient g
    # with dS = Re sum conj(g) dU (the conjugate Wirtinger derivative times 2);
    # then dS = sum Re tr(Mraw dU) for Mraw = g^dag
    g = Ut.grad.detach().numpy()
    Mraw = np.conj(np.swapaxes(g, -1, -2))
    G = -traceless_antihermitian(U @ Mraw)
    return float(S.detach()), Mraw, G


def pf_action_clover(dims, U, kappa, csw, bc, phi, variant="eo", traceless=True, twist=0.0):
    """The action alone (no gradient)."""
    dims = tuple(int(v) for v in dims)
    with torch.no_grad():
        Ut = torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128))
        ph = torch.from_numpy(np.ascontiguousarray(phi, dtype=np.complex128)).reshape(-1)
        return float(_action(Ut, dims, float(kappa), float(csw), bc, traceless, ph, variant, twist))


def _hop_torch(U, psi, bc):
    """(H psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x + mu) + (1 + gamma_mu)
    U_mu(x - mu)^dag psi(x - mu)], with the boundary phase on links that wrap;
    psi [Lt, Lz, Ly, Lx, 4, 3]."""
    g = _gammas()
    one = torch.eye(4, dtype=torch.complex128)
    lt, lz, ly, lx = psi.shape[:4]
    t, z, y, x = torch.meshgrid(torch.arange(lt), torch.arange(lz), torch.arange(ly), torch.arange(lx),
                                indexing="ij")
    coord, ext = [x, y, z, t], [lx, ly, lz, lt]
    out = torch.zeros_like(psi)
    for mu in range(4):
        ph = complex(bc[mu])
        c128 = dict(dtype=torch.complex128)
        phf = torch.where(coord[mu] == ext[mu] - 1, torch.tensor(ph, **c128), torch.tensor(1.0 + 0j, **c128))
        phb = torch.where(coord[mu] == 0, torch.tensor(np.conj(ph), **c128), torch.tensor(1.0 + 0j, **c128))
        u = U[..., mu, :, :]
        f = torch.einsum("...cd,...sd->...sc", u, _fwd(psi, mu)) * phf[..., None, None]
        b = torch.einsum("...cd,...sd->...sc", _h(_bwd(u, mu)), _bwd(psi, mu)) * phb[..., None, None]
        out = out + torch.einsum("st,...tc->...sc", one - g[mu], f) + torch.einsum("st,...tc->...sc", one + g[mu], b)
    return out


def _block_apply(A, psi):
    shape = psi.shape
    return torch.einsum("...ij,...j->...i", A, psi.reshape(*shape[:4], 12)).reshape(shape)


def pf_force_clover_mf(dims, U, kappa, csw, bc, phi, variant="eo", traceless=True, tol=1e-13, twist=0.0):
    """pf_force_clover without dense matrices: (S, Mraw, G) for the even-odd
    or full-lattice clover (or, at c_sw = 0, Wilson; with twist, twisted-mass)
    action."""
    dims = tuple(int(v) for v in dims)
    op = Operator(dims, U, kappa, csw, bc, traceless, twist=twist)
    if variant == "eo":
        X, _ = cg(op.schur_normal, np.ascontiguousarray(phi, dtype=np.complex128), tol)
        Y = op.schur(X)
        Xf, Yf = from_parity(dims, X, 0), from_parity(dims, Y, 0)
    else:
        X, _ = cg(op.DdagD, np.ascontiguousarray(phi, dtype=np.complex128).reshape(op.shape), tol)
        Y = op.D(X)
        Xf, Yf = X, Y
    S = float(np.vdot(np.asarray(phi).reshape(-1), X.reshape(-1)).real)
    Ut = torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128)).clone().requires_grad_(True)
    Xt, Yt = torch.from_numpy(Xf), torch.from_numpy(Yf)
    A = _site_blocks(Ut, dims, float(kappa), float(csw), traceless, twist)
    if variant == "eo":
        # M X = A_ee X - kappa^2 H_eo A_oo^-1 H_oe X with X on the even sites
        odd = torch.from_numpy(np.ascontiguousarray(_parity_mask(dims)))
        Aodd = torch.where(odd[..., None, None], A, torch.eye(12, dtype=torch.complex128))
        t = _hop_torch(Ut, Xt, bc)                  # H_oe X (odd sites)
        t = torch.linalg.solve(Aodd, t.reshape(*t.shape[:4], 12)).reshape(t.shape)
        t = _hop_torch(Ut, t * odd[..., None, None], bc)
        MX = (_block_apply(A, Xt) - float(kappa) ** 2 * t) * (~odd)[..., None, None]
    else:
        MX = _block_apply(A, Xt) - float(kappa) * _hop_torch(Ut, Xt, bc)
    f = (Yt.conj() * MX).real.sum()
    f.backward()
    g = -2.0 * Ut.grad.detach().numpy()
    Mraw = np.conj(np.swapaxes(g, -1, -2))
    G = -traceless_antihermitian(np.asarray(U) @ Mraw)
    return S, Mraw, G


def _parity_mask(dims):
    """True on odd sites, [Lt, Lz, Ly, Lx]."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return ((x + y + z + t) % 2) == 1
