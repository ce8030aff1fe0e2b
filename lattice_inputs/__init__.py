"""Seeded synthetic inputs for the Wilson / Wilson-clover solver path.

This module is shared by the HIP path's tests and benchmark and by the
oracle's tests.  It only draws random numbers and builds input arrays (gauge
links, sources, gauge transformations); it holds none of the fermion-matrix
arithmetic.

Array layouts (C-contiguous, complex128):
  gauge field  U[t, z, y, x, mu, a, b]   mu = 0..3 for x, y, z, t
  spinor     psi[t, z, y, x, spin, colour]   (spin-colour index ic + 3*is)
Lattice dimensions are given as dims = (Lx, Ly, Lz, Lt).
"""
from __future__ import annotations

import numpy as np

LINK_SEED_BASE = 1000
SOURCE_SEED_BASE = 2000


def _shape(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def haar_su3(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-random SU(3) matrices: QR of a complex Gaussian matrix, the
    phases of R's diagonal moved into Q, then Q divided by the principal cube
    root of its determinant so that det = 1."""
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / np.power(det, 1.0 / 3.0)[:, None, None]
    return q


def random_traceless_hermitian(rng: np.random.Generator, n: int) -> np.ndarray:
    """H = (A + A^dag)/2 minus its trace, A with unit-variance Gaussian real
    and imaginary parts."""
    a = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    return h - tr[:, None, None] * np.eye(3)[None]


def expi_traceless_hermitian(q: np.ndarray) -> np.ndarray:
    """exp(i Q) for traceless Hermitian 3x3 Q, in closed form (Morningstar and
    Peardon, Phys. Rev. D 69 (2004) 054501, Sec. III): exp(iQ) = f0 + f1 Q +
    f2 Q^2 with f_j from c0 = det Q and c1 = tr(Q^2)/2; negative c0 is
    mapped to positive by f_j(-c0) = (-1)^j conj(f_j(c0))."""
    q2 = q @ q
    c0 = np.linalg.det(q).real
    c1 = 0.5 * np.trace(q2, axis1=-2, axis2=-1).real
    neg = c0 < 0
    c0a = np.abs(c0)
    c1 = np.maximum(c1, 1e-300)
    c0max = 2.0 * (c1 / 3.0) ** 1.5
    theta = np.arccos(np.clip(c0a / c0max, -1.0, 1.0))
    u = np.sqrt(c1 / 3.0) * np.cos(theta / 3.0)
    w = np.sqrt(c1) * np.sin(theta / 3.0)
    xi0 = np.where(np.abs(w) > 0.05, np.sin(w) / np.where(w == 0, 1, w),
                   1 - w ** 2 / 6 * (1 - w ** 2 / 20 * (1 - w ** 2 / 42)))
    e2iu = np.exp(2j * u)
    emiu = np.exp(-1j * u)
    cw = np.cos(w)
    h0 = (u * u - w * w) * e2iu + emiu * (8 * u * u * cw + 2j * u * (3 * u * u + w * w) * xi0)
    h1 = 2 * u * e2iu - emiu * (2 * u * cw - 1j * (3 * u * u - w * w) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9 * u * u - w * w
    f0, f1, f2 = h0 / den, h1 / den, h2 / den
    f0 = np.where(neg, np.conj(f0), f0)
    f1 = np.where(neg, -np.conj(f1), f1)
    f2 = np.where(neg, np.conj(f2), f2)
    eye = np.eye(3)[None]
    return f0[:, None, None] * eye + f1[:, None, None] * q + f2[:, None, None] * q2


def exp_iH_su3(rng: np.random.Generator, n: int, eps: float, chunk: int = 1 << 20) -> np.ndarray:
    """n matrices U = exp(i*eps*H), H traceless Hermitian built from a complex
    matrix with unit-variance Gaussian real and imaginary parts."""
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        out[s:s + m] = expi_traceless_hermitian(eps * random_traceless_hermitian(rng, m))
    return out


def gauge_haar(dims, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = volume(dims)
    return haar_su3(rng, v * 4).reshape(_shape(dims) + (4, 3, 3))


def gauge_exp(dims, eps: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = volume(dims)
    return exp_iH_su3(rng, v * 4, eps).reshape(_shape(dims) + (4, 3, 3))


def gauge_unit(dims) -> np.ndarray:
    v = volume(dims)
    u = np.zeros((v * 4, 3, 3), dtype=np.complex128)
    u[:, 0, 0] = u[:, 1, 1] = u[:, 2, 2] = 1.0
    return u.reshape(_shape(dims) + (4, 3, 3))


def gauge_abelian_twist(dims, n_flux: int = 1) -> np.ndarray:
    """Constant abelian field strength in the x-y plane: U_y(x) =
    diag(e^{i phi x}, e^{-i phi x}, 1) with phi = 2 pi n_flux / Lx (so the
    field is uniform across the x boundary), all other links unit."""
    lx = int(dims[0])
    phi = 2.0 * np.pi * n_flux / lx
    u = gauge_unit(dims).copy()
    xs = np.arange(lx)
    u[..., 1, 0, 0] = np.exp(1j * phi * xs)[None, None, None, :]
    u[..., 1, 1, 1] = np.exp(-1j * phi * xs)[None, None, None, :]
    return u


def gauge_u1_diag(dims, seed: int, amp: float = 1.0) -> np.ndarray:
    """Diagonal links diag(e^{i a}, e^{i b}, e^{-i(a+b)}) with uniform random
    angles in [-amp*pi, amp*pi] (an abelian U(1)^2 field inside SU(3))."""
    rng = np.random.default_rng(seed)
    v = volume(dims)
    a = rng.uniform(-amp * np.pi, amp * np.pi, size=(v * 4,))
    b = rng.uniform(-amp * np.pi, amp * np.pi, size=(v * 4,))
    u = np.zeros((v * 4, 3, 3), dtype=np.complex128)
    u[:, 0, 0] = np.exp(1j * a)
    u[:, 1, 1] = np.exp(1j * b)
    u[:, 2, 2] = np.exp(-1j * (a + b))
    return u.reshape(_shape(dims) + (4, 3, 3))


def gauge_transform(dims, seed: int) -> np.ndarray:
    """A random SU(3) gauge transformation Omega[t, z, y, x, a, b]."""
    rng = np.random.default_rng(seed)
    return haar_su3(rng, volume(dims)).reshape(_shape(dims) + (3, 3))


def gaussian_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian spinor field (real and imaginary parts i.i.d. N(0,1))."""
    rng = np.random.default_rng(seed)
    shp = _shape(dims) + (4, 3)
    if nrhs is not None:
        shp = (nrhs,) + shp
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def gaussian_parity_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian spinor on one parity: [Vh, 4, 3] (or [nrhs, Vh, 4, 3])."""
    rng = np.random.default_rng(seed)
    shp = (volume(dims) // 2, 4, 3)
    if nrhs is not None:
        shp = (nrhs,) + shp
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def point_sources(dims, site=(0, 0, 0, 0)) -> np.ndarray:
    """The 12 unit point sources at one site, source k = ic + 3*is with a 1 at
    spin is, colour ic: array [12, t, z, y, x, 4, 3]."""
    x, y, z, t = site
    out = np.zeros((12,) + _shape(dims) + (4, 3), dtype=np.complex128)
    for s in range(4):
        for c in range(3):
            out[c + 3 * s, t, z, y, x, s, c] = 1.0
    return out


def random_su3_algebra(dims, seed: int) -> np.ndarray:
    """Random traceless anti-Hermitian 3x3 matrices X_mu(x), one per link:
    X[t, z, y, x, mu, a, b], Gaussian components."""
    rng = np.random.default_rng(seed)
    n = volume(dims) * 4
    a = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    x = 0.5 * (a - np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(x, axis1=-2, axis2=-1) / 3.0
    x = x - tr[:, None, None] * np.eye(3)[None]
    return x.reshape(_shape(dims) + (4, 3, 3))


# Workloads: (name, dims, link generator, kappa, c_sw, boundary phases)
ANTIPERIODIC_T = (1.0 + 0j, 1.0 + 0j, 1.0 + 0j, -1.0 + 0j)

WORKLOADS = {
    "wilson_4x4x4x4": dict(dims=(4, 4, 4, 4), links="haar", eps=None, kappa=0.12, csw=0.0, k=0),
    "clover_16x16x16x32": dict(dims=(16, 16, 16, 32), links="exp", eps=0.3, kappa=0.13, csw=1.0, k=1),
    "clover_32x32x32x64": dict(dims=(32, 32, 32, 64), links="exp", eps=0.5, kappa=0.1355, csw=1.7, k=2),
    "clover_24x24x24x48": dict(dims=(24, 24, 24, 48), links="exp", eps=0.5, kappa=0.135, csw=1.7, k=3),
    "wilson_16x16x16x16": dict(dims=(16, 16, 16, 16), links="exp", eps=0.3, kappa=0.125, csw=0.0, k=4),
}

RAGGED_DIMS = ((8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32), (20, 20, 20, 40))


def workload_gauge(name: str, dims=None) -> np.ndarray:
    w = WORKLOADS[name]
    d = dims if dims is not None else w["dims"]
    seed = LINK_SEED_BASE + w["k"]
    if w["links"] == "haar":
        return gauge_haar(d, seed)
    return gauge_exp(d, w["eps"], seed)


def workload_source(name: str, dims=None, nrhs=None) -> np.ndarray:
    w = WORKLOADS[name]
    d = dims if dims is not None else w["dims"]
    return gaussian_spinor(d, SOURCE_SEED_BASE + w["k"], nrhs)
