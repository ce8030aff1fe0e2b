"""Dense fermion matrix built entry by entry from eq. (1) (Sec. 3) of the
Bridge++ 2.0 paper, for brute-force checks on tiny lattices (2^4, 4^4).

TEST INFRASTRUCTURE ONLY.  This is a second, independent writing of the
operator: it builds its own gamma matrices, computes the clover term from
generic path-ordered products and sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],
and assembles D as an N x N numpy matrix (N = 12 V, index 12*lex + 3*spin +
colour).  It is used to check the matrix-free C oracle, not the HIP path.
"""
from __future__ import annotations

import numpy as np


def chiral_gammas():
    """gamma_1..gamma_4 (x, y, z, t) of the chiral basis and gamma_5."""
    s1 = np.array([[0, 1], [1, 0]], dtype=complex)
    s2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
    s3 = np.array([[1, 0], [0, -1]], dtype=complex)
    z = np.zeros((2, 2), dtype=complex)
    e = np.eye(2, dtype=complex)
    g = [np.block([[z, -1j * s], [1j * s, z]]) for s in (s1, s2, s3)]
    g.append(np.block([[z, e], [e, z]]))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


def _coords(dims):
    lx, ly, lz, lt = dims
    out = []
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    out.append((x, y, z, t))
    return out


def _lex(dims, c):
    lx, ly, lz, lt = dims
    return c[0] + lx * (c[1] + ly * (c[2] + lz * c[3]))


def _shift(dims, c, mu, d):
    c = list(c)
    c[mu] += d
    wrapped = c[mu] < 0 or c[mu] >= dims[mu]
    c[mu] %= dims[mu]
    return tuple(c), wrapped


def _link(U, dims, c, mu):
    x, y, z, t = c
    return U[t, z, y, x, mu]


def path_product(U, dims, c, steps):
    """Ordered product of links along a path that starts at c; a step +mu
    uses U_mu(here), a step -mu uses U_mu(here - mu)^dag."""
    m = np.eye(3, dtype=complex)
    here = tuple(c)
    for st in steps:
        mu = abs(st) - 1
        if st > 0:
            m = m @ _link(U, dims, here, mu)
            here, _ = _shift(dims, here, mu, +1)
        else:
            there, _ = _shift(dims, here, mu, -1)
            m = m @ _link(U, dims, there, mu).conj().T
            here = there
    assert here == tuple(c), "path is not closed"
    return m


def clover_site(U, dims, c, csw, kappa, traceless=True):
    """F(x) = i c_sw kappa sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}, with
    Fhat = (Q - Q^dag)/8 and Q the four counter-clockwise leaves."""
    g, _ = chiral_gammas()
    F = np.zeros((12, 12), dtype=complex)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            m, n = mu + 1, nu + 1
            leaves = ([m, n, -m, -n], [n, -m, -n, m], [-m, -n, m, n], [-n, m, n, -m])
            Q = sum(path_product(U, dims, c, lf) for lf in leaves)
            Fh = (Q - Q.conj().T) / 8.0
            if traceless:
                Fh = Fh - np.trace(Fh) / 3.0 * np.eye(3)
            sigma = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
            F += 1j * csw * kappa * np.kron(sigma, Fh)
    return F


def dense_dirac(dims, U, kappa, csw=0.0, bc=(1, 1, 1, 1), traceless=True, twist=0.0):
    """The N x N matrix D of eq. (1); blocks are kron(spin 4x4, colour 3x3).
    twist != 0 adds the twisted-mass term i twist gamma_5 on every site."""
    dims = tuple(int(v) for v in dims)
    g, g5 = chiral_gammas()
    V = int(np.prod(dims))
    N = 12 * V
    D = np.zeros((N, N), dtype=complex)
    one = np.eye(4, dtype=complex)
    for c in _coords(dims):
        i = _lex(dims, c)
        bi = slice(12 * i, 12 * i + 12)
        D[bi, bi] += np.eye(12)
        if twist != 0.0:
            D[bi, bi] += 1j * twist * np.kron(g5, np.eye(3))
        if csw != 0.0:
            D[bi, bi] += clover_site(U, dims, c, csw, kappa, traceless)
        for mu in range(4):
            y, w = _shift(dims, c, mu, +1)
            ph = complex(bc[mu]) if w else 1.0
            j = _lex(dims, y)
            D[bi, 12 * j:12 * j + 12] += -kappa * ph * np.kron(one - g[mu], _link(U, dims, c, mu))
            y, w = _shift(dims, c, mu, -1)
            ph = np.conj(complex(bc[mu])) if w else 1.0
            j = _lex(dims, y)
            D[bi, 12 * j:12 * j + 12] += -kappa * ph * np.kron(one + g[mu], _link(U, dims, y, mu).conj().T)
    return D


def parity_index(dims, p):
    """Dense-vector indices of all components on parity p, in checkerboard order."""
    idx = []
    for c in _coords(dims):
        if sum(c) % 2 == p:
            i = _lex(dims, c)
            idx.extend(range(12 * i, 12 * i + 12))
    return np.asarray(idx)
