"""Oracle of the two-level multigrid pieces: the aggregation prolongator and
the Galerkin coarse operator (Sec. 1 cites adaptive multigrid for lattice
QCD and Sec. 4 lists multigrid among the solvers; the construction is read
as adaptive aggregation: near-null vectors split by chirality, orthonormal
per aggregate, coarse operator P^dag D P).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Conventions: fields [Lt, Lz, Ly, Lx, 4, 3] as in the oracle; aggregates are
blocks of block = (bx, by, bz, bt) sites, numbered lexicographically over the
coarse lattice (L / block) with x fastest; the coarse degrees of freedom of
aggregate A are r = chi * nvec + k (chirality chi: spins 0, 1 or 2, 3;
vector k); a coarse vector is [ncoarse, 2 nvec].  The coarse stencil holds
for each aggregate A nine blocks D_c[A][d]: d = 0 couples A to itself,
d = 1 + 2 mu to the aggregate at +mu, d = 2 + 2 mu to the one at -mu.
"""
from __future__ import annotations

import numpy as np


def coarse_dims(dims, block):
    return tuple(int(L) // int(b) for L, b in zip(dims, block))


def aggregate_map(dims, block) -> np.ndarray:
    """Aggregate index of every site, as an array [Lt, Lz, Ly, Lx]."""
    Lx, Ly, Lz, Lt = dims
    cx, cy, cz, ct = coarse_dims(dims, block)
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    ax, ay, az, at = x // block[0], y // block[1], z // block[2], t // block[3]
    return ax + cx * (ay + cy * (az + cz * at))


def block_orthonormalize(dims, block, V) -> np.ndarray:
    """Per aggregate and chirality, modified Gram-Schmidt of the vectors
    V[k] (k in order): v_k -= <v_j, v_k> v_j for j < k, then v_k /= |v_k|,
    with inner products over the aggregate's sites and the chirality's two
    spins and three colours.  A vanishing part is left zero."""
    W = np.array(V, dtype=np.complex128, copy=True)
    agg = aggregate_map(dims, block)
    nagg = int(agg.max()) + 1
    for A in range(nagg):
        mask = agg == A
        for chi in range(2):
            sl = slice(2 * chi, 2 * chi + 2)
            parts = [W[k][mask][:, sl, :].reshape(-1).copy() for k in range(len(W))]
            for k in range(len(W)):
                for j in range(k):
                    parts[k] = parts[k] - np.vdot(parts[j], parts[k]) * parts[j]
                n = np.linalg.norm(parts[k])
                if n > 0:
                    parts[k] = parts[k] / n
            for k in range(len(W)):
                sub = W[k][mask]
                sub[:, sl, :] = parts[k].reshape(sub[:, sl, :].shape)
                W[k][mask] = sub
    return W


def prolongator(dims, block, W) -> np.ndarray:
    """Dense P [12 V, ncoarse * 2 nvec]: column A * 2 nvec + chi * nvec + k is
    the chirality-chi part of W[k] on aggregate A (zero elsewhere); rows in
    the oracle's field order (site lexicographic, then spin, colour)."""
    nv = len(W)
    agg = aggregate_map(dims, block).reshape(-1)
    nagg = int(agg.max()) + 1
    V = agg.size
    P = np.zeros((V * 12, nagg * 2 * nv), dtype=np.complex128)
    for k in range(nv):
        w = W[k].reshape(V, 4, 3)
        for chi in range(2):
            part = np.zeros_like(w)
            part[:, 2 * chi:2 * chi + 2, :] = w[:, 2 * chi:2 * chi + 2, :]
            for A in range(nagg):
                col = A * 2 * nv + chi * nv + k
                m = agg == A
                field = np.zeros_like(w)
                field[m] = part[m]
                P[:, col] = field.reshape(-1)
    return P


def restrict(P, f) -> np.ndarray:
    """P^dag f as a coarse vector (flat)."""
    return P.conj().T @ np.asarray(f).reshape(-1)


def prolong(P, c) -> np.ndarray:
    return P @ np.asarray(c).reshape(-1)


def galerkin(D, P) -> np.ndarray:
    """The coarse operator P^dag D P from a dense fine operator D."""
    return P.conj().T @ (D @ P)


def neighbour(cdims, A, d) -> int:
    """Aggregate reached from A by stencil direction d (0: A itself)."""
    a = []
    r = A
    for L in cdims:
        a.append(r % L)
        r //= L
    if d > 0:
        mu = (d - 1) // 2
        a[mu] = (a[mu] + (1 if d % 2 == 1 else -1)) % cdims[mu]
    return a[0] + cdims[0] * (a[1] + cdims[1] * (a[2] + cdims[2] * a[3]))


def stencil_to_dense(cdims, Dc) -> np.ndarray:
    """Dense coarse matrix from stencil blocks Dc [ncoarse, 9, n2, n2] (blocks
    of directions reaching the same aggregate add up)."""
    nagg, _, n2, _ = Dc.shape
    M = np.zeros((nagg * n2, nagg * n2), dtype=np.complex128)
    for A in range(nagg):
        for d in range(9):
            B = neighbour(cdims, A, d)
            M[A * n2:(A + 1) * n2, B * n2:(B + 1) * n2] += Dc[A, d]
    return M


def coarse_columns(apply_D, dims, block, W, A0) -> np.ndarray:
    """Block column A0 of P^dag D P, matrix-free: for each coarse degree of
    freedom c of aggregate A0, the restriction of D applied to the column
    (P e_c).  Returns [ncoarse, n2 (rows), n2 (columns c)]."""
    nv = len(W)
    agg = aggregate_map(dims, block)
    nagg = int(agg.max()) + 1
    n2 = 2 * nv
    out = np.zeros((nagg, n2, n2), dtype=np.complex128)
    Wf = np.asarray(W)
    for c in range(n2):
        chi, k = divmod(c, nv)
        col = np.zeros_like(Wf[0])
        m = agg == A0
        col[m, 2 * chi:2 * chi + 2, :] = Wf[k][m, 2 * chi:2 * chi + 2, :]
        y = apply_D(col)
        for A in range(nagg):
            mA = agg == A
            for r in range(n2):
                rchi, rk = divmod(r, nv)
                out[A, r, c] = np.vdot(Wf[rk][mA][:, 2 * rchi:2 * rchi + 2, :], y[mA][:, 2 * rchi:2 * rchi + 2, :])
    return out
