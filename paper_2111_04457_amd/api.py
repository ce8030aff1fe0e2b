"""Python binding of the C ABI (include/lq.h): argument marshalling only.

Every computation runs in the HIP library; torch supplies device memory
(complex128 CUDA tensors) and the current stream.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check, load


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _bc_array(bc):
    if bc is None:
        bc = (1, 1, 1, 1)
    arr = ((ctypes.c_double * 2) * 4)()
    for i, v in enumerate(bc):
        v = complex(*v) if isinstance(v, (tuple, list)) else complex(v)
        arr[i][0] = v.real
        arr[i][1] = v.imag
    return arr


def _dev(t: torch.Tensor, shape, name, host_ok: bool = False):
    """t as a contiguous complex128 tensor of trailing shape `shape`, on the
    GPU (or, with host_ok, in host memory: the *_host entry points)."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or \
            not (t.device.type == "cuda" or (host_ok and t.device.type == "cpu")):
        raise TypeError("%s must be a complex128 %s tensor" % (name, "CUDA or CPU" if host_ok else "CUDA"))
    if tuple(t.shape[-len(shape):]) != tuple(shape):
        raise ValueError("%s has shape %s, expected [..., %s]" % (name, tuple(t.shape), shape))
    return t.contiguous()


def _op_params(dims, kappa, csw=0.0, bc=None, traceless=True, link_recon=18, twist=0.0) -> _lib.OpParams:
    p = _lib.OpParams()
    load().lq_op_params_default(ctypes.byref(p))
    for i in range(4):
        p.dims[i] = int(dims[i])
    p.kappa = float(kappa)
    p.csw = float(csw)
    p.bc = _bc_array(bc)
    p.clover_traceless = int(bool(traceless))
    p.link_recon = int(link_recon)
    p.twist = float(twist)
    return p


def workspace_bytes(dims, csw=0.0, link_recon=18, nrhs: int = 1) -> int:
    """Bytes of the device workspace an operator of this lattice needs for
    calls of up to nrhs right-hand sides (lq_workspace_bytes; no GPU needed)."""
    n = ctypes.c_size_t()
    check(load().lq_workspace_bytes(ctypes.byref(_op_params(dims, 0.125, csw, None, True, link_recon)), int(nrhs),
                                    ctypes.byref(n)))
    return n.value


@dataclass
class SolverParams:
    """params_solver of the paper's Fig. 1."""
    solver: str = "bicgstab"     # "bicgstab" | "cgne"
    tol: float = 1e-10           # true relative residual |b - D x| / |b|
    max_iter: int = 100000
    inner: str = "f32"           # "f64" (plain FP64 solve), "f32", "f16"
    inner_tol: float = 1e-5
    max_outer: int = 100
    check_every: int = 8
    even_odd: bool = True
    left_precond: bool = False   # inner BiCGStab on A_ee^-1 M (clover, even-odd)
    reliable: bool = False       # keep the inner Krylov space across FP64 residual replacements
    deflate: bool = False        # project each outer residual with the operator's deflation space

    def to_c(self) -> _lib.SolverParams:
        p = _lib.SolverParams()
        load().lq_solver_params_default(ctypes.byref(p))
        p.solver = {"cgne": _lib.CGNE, "bicgstab": _lib.BICGSTAB}[self.solver]
        p.tol = self.tol
        p.max_iter = self.max_iter
        p.inner = _lib.PREC[self.inner]
        p.inner_tol = self.inner_tol
        p.max_outer = self.max_outer
        p.check_every = self.check_every
        p.even_odd = int(bool(self.even_odd))
        p.left_precond = int(bool(self.left_precond))
        p.reliable = int(bool(self.reliable))
        p.deflate = int(bool(self.deflate))
        return p


@dataclass
class SolveStats:
    nconv: int
    nouter: int
    restarts: int
    converged: bool
    diff: float
    t_solve_ms: float
    hop_bytes: float
    n_hop: int


class Operator:
    """The fermion matrix of eq. (1) on one gauge field (params_fopr +
    set_config of Fig. 1)."""

    def __init__(self, dims, kappa, csw=0.0, bc=None, traceless=True, link_recon=18, twist=0.0):
        lib = load()
        p = _op_params(dims, kappa, csw, bc, traceless, link_recon, twist)
        h = ctypes.c_void_p()
        check(lib.lq_op_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._ws = None  # the bound workspace (a torch uint8 tensor), if any
        self.dims = tuple(int(d) for d in dims)
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.full_shape = tuple(self.dims[::-1]) + (4, 3)
        self.parity_shape = (self.V // 2, 4, 3)

    def close(self):
        if getattr(self, "_h", None):
            load().lq_op_destroy(self._h)
            self._h = None
        self._ws = None

    def workspace_bytes(self, nrhs: int = 1) -> int:
        n = ctypes.c_size_t()
        check(load().lq_op_workspace_bytes(self._h, int(nrhs), ctypes.byref(n)))
        return n.value

    def bind(self, nrhs: int = 1) -> torch.Tensor:
        """Allocate the operator's device memory as one torch tensor (uint8,
        lq_op_workspace_bytes(nrhs) bytes) and bind it (lq_op_bind): from
        then on the library allocates no device memory for set_gauge, apply
        and solve.  Drops the gauge field (set it again).  Returns the tensor."""
        ws = torch.empty(self.workspace_bytes(nrhs), dtype=torch.uint8, device="cuda")
        check(load().lq_op_bind(self._h, ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        self._ws = ws
        return ws

    def unbind(self):
        """Give the device memory back to the library's own allocations."""
        check(load().lq_op_bind(self._h, None, 0))
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_gauge(self, U: torch.Tensor):
        """U on the GPU (lq_op_set_gauge) or in host memory (lq_op_set_gauge_host)."""
        U = _dev(U, self.dims[::-1] + (4, 3, 3), "U", host_ok=True)
        fn = load().lq_op_set_gauge if U.is_cuda else load().lq_op_set_gauge_host
        check(fn(self._h, ctypes.c_void_p(U.data_ptr()), _stream()))

    def set_params(self, kappa, csw, bc=None):
        arr = None if bc is None else _bc_array(bc)
        check(load().lq_op_set_params(self._h, float(kappa), float(csw),
                                      None if arr is None else ctypes.byref(arr), _stream()))

    def apply(self, kind: str, psi: torch.Tensor, prec: str = "f64") -> torch.Tensor:
        """out = K psi for K in D, Ddag, DdagD (full fields) or the parity kinds;
        psi on the GPU (lq_op_apply) or in host memory (lq_op_apply_host, the
        result then in host memory too)."""
        full = kind in _lib.FULL_KINDS
        shape = self.full_shape if full else self.parity_shape
        psi = _dev(psi, shape, "psi", host_ok=True)
        nrhs = psi.numel() // (12 * (self.V if full else self.V // 2))
        out = torch.empty_like(psi)
        fn = load().lq_op_apply if psi.is_cuda else load().lq_op_apply_host
        check(fn(self._h, _lib.KINDS[kind], _lib.PREC[prec], ctypes.c_void_p(out.data_ptr()),
                 ctypes.c_void_p(psi.data_ptr()), nrhs, _stream()))
        return out

    def apply_noalloc(self, kind: str, psi: torch.Tensor, out: torch.Tensor, prec: str = "f64") -> torch.Tensor:
        """out = K psi like apply(), through lq_op_apply_noalloc: the library
        allocates nothing (its packed fields use a fixed per-GPU array); out
        is the caller's tensor of psi's shape."""
        full = kind in _lib.FULL_KINDS
        shape = self.full_shape if full else self.parity_shape
        psi = _dev(psi, shape, "psi")
        if not (isinstance(out, torch.Tensor) and out.dtype == torch.complex128 and out.is_cuda
                and out.is_contiguous() and out.shape == psi.shape):
            raise ValueError("out must be a contiguous complex128 CUDA tensor of psi's shape")
        nrhs = psi.numel() // (12 * (self.V if full else self.V // 2))
        check(load().lq_op_apply_noalloc(self._h, _lib.KINDS[kind], _lib.PREC[prec], ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(psi.data_ptr()), nrhs, _stream()))
        return out

    def traffic(self, prec="f32", nrhs=1, clover=False):
        b = ctypes.c_double()
        f = ctypes.c_double()
        check(load().lq_op_traffic(self._h, _lib.PREC[prec], int(nrhs), int(bool(clover)), ctypes.byref(b),
                                   ctypes.byref(f)))
        return b.value, f.value

    def set_option(self, name: str, value: int):
        check(load().lq_op_set_option(self._h, name.encode(), int(value)))

    def get_option(self, name: str) -> int:
        v = ctypes.c_int()
        check(load().lq_op_get_option(self._h, name.encode(), ctypes.byref(v)))
        return v.value

    def set_block(self, prec: str, block: int):
        check(load().lq_op_set_block(self._h, _lib.PREC[prec], int(block)))

    def eigs(self, nev: int = 8, m: int = 64, v0: torch.Tensor | None = None, tol: float = 1e-8,
             vectors: bool = False, seed: int = 0, max_restarts: int = 100, cheb_degree: int = 8,
             cheb_lo: float = 0.0, cheb_hi: float = 0.0):
        """The nev smallest eigenvalues of M^dag M (lq_eigs: thick-restart
        Lanczos with full reorthogonalisation, m basis vectors per cycle, on
        M^dag M or on its Chebyshev filter of degree cheb_degree over
        [cheb_lo, cheb_hi], 0 = automatic).  Returns (evals, resid, evecs or
        None, stats dict); v0 defaults to a seeded Gaussian even field."""
        if v0 is None:
            gen = torch.Generator(device="cpu").manual_seed(seed)
            v0 = torch.randn(self.parity_shape + (2,), generator=gen, dtype=torch.float64)
            v0 = torch.view_as_complex(v0).cuda()
        v0 = _dev(v0, self.parity_shape, "v0")
        p = _lib.EigParams()
        load().lq_eig_params_default(ctypes.byref(p))
        p.nev, p.m, p.max_restarts, p.cheb_degree = int(nev), int(m), int(max_restarts), int(cheb_degree)
        p.cheb_lo, p.cheb_hi, p.tol = float(cheb_lo), float(cheb_hi), float(tol)
        ev = (ctypes.c_double * nev)()
        rs = (ctypes.c_double * nev)()
        st = _lib.EigStats()
        X = torch.empty((nev,) + self.parity_shape, dtype=torch.complex128, device="cuda") if vectors else None
        rc = load().lq_eigs(self._h, ctypes.byref(p), ctypes.c_void_p(v0.data_ptr()), ev, rs,
                            ctypes.c_void_p(X.data_ptr()) if X is not None else None, ctypes.byref(st), _stream())
        check(rc, allow_not_converged=True)
        stats = {"nconv": st.nconv, "restarts": st.restarts, "applies": st.applies, "cheb_lo": st.cheb_lo,
                 "cheb_hi": st.cheb_hi}
        return list(ev), list(rs), X, stats

    def deflated_guess(self, b: torch.Tensor, evals, evecs: torch.Tensor) -> torch.Tensor:
        """The initial guess of lq_deflated_guess for D x = b: the even-odd
        solution's component in the span of the eigenvectors evecs
        ([nvec, Lt/2.., 4, 3] even fields, as eigs returns them) of M^dag M
        with eigenvalues evals, and the odd half that satisfies the odd
        rows.  Pass it to solve(..., x0=...)."""
        b = _dev(b, self.full_shape, "b")
        nvec = len(evals)
        evecs = _dev(evecs, self.parity_shape, "evecs")
        if b.numel() != 12 * self.V or evecs.numel() != nvec * 6 * self.V:
            raise ValueError("deflated_guess takes one right-hand side and one even field per eigenvalue")
        ev = (ctypes.c_double * nvec)(*[float(e) for e in evals])
        x0 = torch.empty_like(b)
        check(load().lq_deflated_guess(self._h, nvec, ev, ctypes.c_void_p(evecs.data_ptr()),
                                       ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x0.data_ptr()), _stream()))
        return x0

    def set_deflation(self, evals, evecs: torch.Tensor | None) -> None:
        """Give the operator's solves (SolverParams(deflate=True)) the
        deflation space of lq_op_set_deflation: eigenpairs of M^dag M as eigs
        returns them (evecs [nvec, V/2, 4, 3]: even fields in checkerboard
        order, on the device); an empty evals removes it."""
        nvec = len(evals) if evecs is not None else 0
        if nvec == 0:
            check(load().lq_op_set_deflation(self._h, 0, None, None, _stream()))
            return
        evecs = _dev(evecs, self.parity_shape, "evecs")
        if evecs.numel() != nvec * 6 * self.V:
            raise ValueError("set_deflation takes one even field per eigenvalue")
        ev = (ctypes.c_double * nvec)(*[float(e) for e in evals])
        check(load().lq_op_set_deflation(self._h, nvec, ev, ctypes.c_void_p(evecs.data_ptr()), _stream()))

    def tune(self, nrhs: int = 1, cache: str | None = None, left: bool = False) -> dict:
        """Autotune the hopping kernels (lq_tune) on the operator form the
        solver will run (left: the A_ee^-1-preconditioned inner system of
        left_precond); returns the JSON report."""
        import json
        self.set_option("tune_form", int(bool(left)))
        buf = ctypes.create_string_buffer(4096)
        check(load().lq_tune(self._h, int(nrhs), cache.encode() if cache else None, buf, len(buf), _stream()))
        return json.loads(buf.value.decode())

    def solve(self, b: torch.Tensor, mode: str = "D", params: SolverParams | None = None,
              x0: torch.Tensor | None = None):
        """x = mode^-1 b for mode D, Ddag or DdagD (invert of Fig. 1).
        b: [nrhs?, Lt, Lz, Ly, Lx, 4, 3] complex128 on the GPU (lq_solve) or in
        host memory (lq_solve_host; x then in host memory too).  Returns
        (x, [SolveStats])."""
        params = params or SolverParams()
        b = _dev(b, self.full_shape, "b", host_ok=True)
        nrhs = b.numel() // (12 * self.V)
        if x0 is not None:
            x = _dev(x0, self.full_shape, "x0", host_ok=True).to(b.device).clone()
        else:
            x = torch.empty_like(b)  # not read without a guess; every entry is written
        stats = (_lib.SolveStats * nrhs)()
        cp = params.to_c()
        fn = load().lq_solve if b.is_cuda else load().lq_solve_host
        st = fn(self._h, ctypes.byref(cp), _lib.KINDS[mode], nrhs, ctypes.c_void_p(x.data_ptr()),
                ctypes.c_void_p(b.data_ptr()), int(x0 is not None), stats, _stream())
        check(st, allow_not_converged=True)
        out = [SolveStats(s.nconv, s.nouter, s.restarts, bool(s.converged), s.diff, s.t_solve_ms, s.hop_bytes, s.n_hop)
               for s in stats]
        return x, out


def bandwidth_probe(nbytes: int = 1 << 30, mode: str = "copy", reps: int = 10) -> float:
    """GB/s of the library's copy (bytes read + written) or read-only probe
    kernel over nbytes of device memory (lq_bandwidth_probe)."""
    nbytes = int(nbytes) // 16 * 16
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda") if mode == "copy" else None
    us = ctypes.c_double()
    check(load().lq_bandwidth_probe(0 if mode == "copy" else 1, ctypes.c_void_p(dst.data_ptr()) if dst is not None
                                    else None, ctypes.c_void_p(src.data_ptr()), nbytes, int(reps), ctypes.byref(us),
                                    _stream()))
    moved = nbytes * (2 if mode == "copy" else 1)
    return moved / (us.value * 1e-6) / 1e9


class Field:
    """A device-resident parity spinor field in the library's packed layout."""

    def __init__(self, op: Operator, prec: str = "f32", nrhs: int = 1):
        h = ctypes.c_void_p()
        check(load().lq_field_create(op.handle, _lib.PREC[prec], int(nrhs), ctypes.byref(h)))
        self._h = h
        self.op = op
        self.prec = prec
        self.nrhs = nrhs

    def close(self):
        if getattr(self, "_h", None):
            load().lq_field_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def load(self, src: torch.Tensor):
        src = _dev(src, self.op.parity_shape, "src")
        if src.numel() != self.nrhs * 12 * (self.op.V // 2):
            raise ValueError("src holds a different number of right-hand sides")
        check(load().lq_field_import(self._h, ctypes.c_void_p(src.data_ptr()), _stream()))

    def read(self) -> torch.Tensor:
        out = torch.empty((self.nrhs,) + self.op.parity_shape, dtype=torch.complex128, device="cuda")
        check(load().lq_field_export(self._h, ctypes.c_void_p(out.data_ptr()), _stream()))
        return out if self.nrhs > 1 else out[0]


def apply_field(op: Operator, kind: str, out: Field, inp: Field):
    check(load().lq_op_apply_field(op.handle, _lib.KINDS[kind], out.handle, inp.handle, _stream()))


def pf_force(op: Operator, phi: torch.Tensor, params: SolverParams | None = None, variant: str = "eo",
             force_prec: str = "f64", want_x: bool = False):
    """Pseudofermion action and force on the operator's gauge field.
    variant "eo": S = phi^dag (M^dag M)^-1 phi with phi on even sites [V/2, 4, 3];
    "full": S = phi^dag (D^dag D)^-1 phi with phi a full field.
    Returns (S, grad_U, G, X, stats): grad_U the torch-convention gradient
    dS/dU, G = -TA(U M) the su(3) force, X = (A)^-1 phi if want_x."""
    params = params or SolverParams(tol=1e-12, inner="f64", solver="cgne")
    shape = op.parity_shape if variant == "eo" else op.full_shape
    phi = _dev(phi, shape, "phi")
    gshape = tuple(op.dims[::-1]) + (4, 3, 3)
    grad = torch.empty(gshape, dtype=torch.complex128, device="cuda")
    G = torch.empty_like(grad)
    X = torch.empty_like(phi) if want_x else None
    S = ctypes.c_double()
    st = _lib.SolveStats()
    cp = params.to_c()
    rc = load().lq_pf_force(op.handle, ctypes.byref(cp), 0 if variant == "eo" else 1, _lib.PREC[force_prec],
                            ctypes.c_void_p(phi.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                            ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(X.data_ptr()) if X is not None else None,
                            ctypes.byref(S), ctypes.byref(st), _stream())
    check(rc, allow_not_converged=True)
    stats = SolveStats(st.nconv, st.nouter, st.restarts, bool(st.converged), st.diff, st.t_solve_ms, st.hop_bytes,
                       st.n_hop)
    return S.value, grad, G, X, stats


class PseudofermionAction(torch.autograd.Function):
    """S(U, phi) = phi^dag (M^dag M)^-1 phi (Wilson or Wilson-clover, even-odd) or
    phi^dag (D^dag D)^-1 phi (variant "full") as a differentiable function.

    The forward pass loads U into the operator and runs one solve and the
    hand-written force kernel (lq_pf_force), which yields S, dS/dU and
    X = (M^dag M)^-1 phi together; backward scales them by the incoming
    gradient: dS/dU as computed, dS/dphi = 2 X (S is real)."""

    @staticmethod
    def forward(ctx, U, phi, op, params=None, variant="eo", force_prec="f64"):
        op.set_gauge(U)
        S, grad_U, _, X, _ = pf_force(op, phi, params, variant, force_prec, want_x=True)
        ctx.save_for_backward(grad_U, X)
        return torch.tensor(S, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, gS):
        grad_U, X = ctx.saved_tensors
        return gS * grad_U, 2.0 * gS * X, None, None, None, None


class Batch:
    """A ragged batch: several operators (lattices of different volumes),
    nrhs[i] right-hand sides each, solved together (lq_batch_solve)."""

    def __init__(self, ops, nrhs):
        self.ops = list(ops)
        self.nrhs = [int(n) for n in nrhs]
        arr = (ctypes.c_void_p * len(self.ops))(*[o.handle for o in self.ops])
        nr = (ctypes.c_int * len(self.ops))(*self.nrhs)
        h = ctypes.c_void_p()
        check(load().lq_batch_create(arr, len(self.ops), nr, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().lq_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, bs, params: SolverParams | None = None):
        """bs[i]: [nrhs[i], Lt, Lz, Ly, Lx, 4, 3] complex128 CUDA tensors.
        Returns ([x_i], [SolveStats] in batch order)."""
        params = params or SolverParams()
        bs = [_dev(b, op.full_shape, "b").reshape((n,) + op.full_shape) for b, op, n in zip(bs, self.ops, self.nrhs)]
        xs = [torch.zeros_like(b) for b in bs]
        total = sum(self.nrhs)
        stats = (_lib.SolveStats * total)()
        xa = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        ba = (ctypes.c_void_p * len(bs))(*[b.data_ptr() for b in bs])
        cp = params.to_c()
        check(load().lq_batch_solve(self._h, ctypes.byref(cp), xa, ba, stats, _stream()), allow_not_converged=True)
        out = [SolveStats(s.nconv, s.nouter, s.restarts, bool(s.converged), s.diff, s.t_solve_ms, s.hop_bytes, s.n_hop)
               for s in stats]
        return xs, out


@dataclass
class MGParams:
    """Two-level multigrid parameters (lq_mg_params)."""
    block: tuple = (4, 4, 4, 4)   # aggregate extents (x, y, z, t)
    nvec: int = 12                # near-null vectors (coarse dof per aggregate 2 nvec)
    setup_iters: int = 3          # inverse iterations per vector
    setup_tol: float = 1e-2
    smooth_steps: int = 8         # minimal-residual post-smoothing steps
    coarse_tol: float = 0.2
    coarse_max_iter: int = 200
    gcr_restart: int = 16

    def to_c(self) -> _lib.MGParams:
        p = _lib.MGParams()
        load().lq_mg_params_default(ctypes.byref(p))
        for i in range(4):
            p.block[i] = int(self.block[i])
        p.nvec = self.nvec
        p.setup_iters = self.setup_iters
        p.setup_tol = self.setup_tol
        p.smooth_steps = self.smooth_steps
        p.coarse_tol = self.coarse_tol
        p.coarse_max_iter = self.coarse_max_iter
        p.gcr_restart = self.gcr_restart
        return p


class Multigrid:
    """Two-level multigrid for D x = b on an operator (lq_mg_*): v0 are the
    caller's random start vectors [nvec, Lt, Lz, Ly, Lx, 4, 3] (complex128,
    CUDA) of the near-null vector setup."""

    def __init__(self, op: Operator, v0: torch.Tensor, params: MGParams | None = None):
        self.op = op
        self.params = params or MGParams()
        v0 = _dev(v0, op.full_shape, "v0")
        if v0.numel() != self.params.nvec * 12 * op.V:
            raise ValueError("v0 must hold nvec full fields")
        cp = self.params.to_c()
        h = ctypes.c_void_p()
        check(load().lq_mg_create(op.handle, ctypes.byref(cp), ctypes.c_void_p(v0.data_ptr()), ctypes.byref(h),
                                  _stream()))
        self._h = h
        self.ncoarse = 1
        for L, b in zip(op.dims, self.params.block):
            self.ncoarse *= L // b
        self.n2 = 2 * self.params.nvec

    def close(self):
        if getattr(self, "_h", None):
            load().lq_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b: torch.Tensor, params: SolverParams | None = None):
        """x = D^-1 b (one right-hand side [Lt, Lz, Ly, Lx, 4, 3]); returns (x, SolveStats)."""
        params = params or SolverParams()
        b = _dev(b, self.op.full_shape, "b")
        if b.numel() != 12 * self.op.V:
            raise ValueError("Multigrid.solve takes one right-hand side")
        x = torch.empty_like(b)
        st = _lib.SolveStats()
        cp = params.to_c()
        check(load().lq_mg_solve(self._h, ctypes.byref(cp), ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(b.data_ptr()), ctypes.byref(st), _stream()), allow_not_converged=True)
        return x, SolveStats(st.nconv, st.nouter, st.restarts, bool(st.converged), st.diff, st.t_solve_ms,
                             st.hop_bytes, st.n_hop)

    def vectors(self) -> torch.Tensor:
        """The orthonormalised near-null vectors [nvec, Lt, Lz, Ly, Lx, 4, 3]."""
        out = torch.empty((self.params.nvec,) + self.op.full_shape, dtype=torch.complex128, device="cuda")
        check(load().lq_mg_vectors(self._h, ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def coarse_op(self):
        """The coarse operator as a numpy array [ncoarse, 9, 2 nvec, 2 nvec] (complex128)."""
        import numpy as np
        out = np.zeros((self.ncoarse, 9, self.n2, self.n2), dtype=np.complex128)
        check(load().lq_mg_coarse_op(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def restrict(self, f: torch.Tensor) -> torch.Tensor:
        f = _dev(f, self.op.full_shape, "f")
        out = torch.empty((self.ncoarse, self.n2), dtype=torch.complex128, device="cuda")
        check(load().lq_mg_restrict(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    _stream()))
        return out

    def prolong(self, c: torch.Tensor) -> torch.Tensor:
        c = _dev(c, (self.ncoarse, self.n2), "c")
        out = torch.empty(self.op.full_shape, dtype=torch.complex128, device="cuda")
        check(load().lq_mg_prolong(self._h, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   _stream()))
        return out

    def coarse_apply(self, x: torch.Tensor) -> torch.Tensor:
        x = _dev(x, (self.ncoarse, self.n2), "x")
        out = torch.empty_like(x)
        check(load().lq_mg_coarse_apply(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        _stream()))
        return out


@dataclass
class MDParams:
    """Molecular-dynamics parameters (lq_md_params)."""
    beta: float = 5.6
    tau: float = 1.0
    nsteps: int = 10
    integrator: str = "leapfrog"     # or "omelyan"
    lam: float = 0.1931833275037836
    fermion: bool = True
    force_prec: str = "f64"
    chrono: int = 2                  # initial guesses: 0 zero, 1 last solution, 2 linear extrapolation

    def to_c(self):
        p = _lib.MDParams()
        p.beta = float(self.beta)
        p.tau = float(self.tau)
        p.nsteps = int(self.nsteps)
        p.integrator = _lib.INTEGRATORS[self.integrator]
        p.lam = float(self.lam)
        p.fermion = int(bool(self.fermion))
        p.force_prec = _lib.PREC[self.force_prec]
        p.chrono = int(self.chrono)
        return p


@dataclass
class MDStats:
    H0: float
    H1: float
    dH: float
    T0: float
    T1: float
    Sg0: float
    Sg1: float
    Sf0: float
    Sf1: float
    n_force: int
    converged: bool
    iters: int
    t_ms: float


def gauge_force(op: Operator, beta: float, want_force: bool = True):
    """Wilson gauge action S_g and its su(3) force G on the operator's gauge
    field.  Returns (S_g, G or None)."""
    G = torch.empty(tuple(op.dims[::-1]) + (4, 3, 3), dtype=torch.complex128, device="cuda") if want_force else None
    S = ctypes.c_double()
    check(load().lq_gauge_force(op.handle, float(beta), ctypes.c_void_p(G.data_ptr()) if G is not None else None,
                                ctypes.byref(S), _stream()))
    return S.value, G


def md_trajectory(op: Operator, U: torch.Tensor, P: torch.Tensor, phi: torch.Tensor | None, md: MDParams,
                  params: SolverParams | None = None) -> MDStats:
    """One molecular-dynamics trajectory; U and P (complex128 CUDA tensors
    [Lt, Lz, Ly, Lx, 4, 3, 3]) are updated in place, and the operator holds
    the final U.  phi: even-site pseudofermion [V/2, 4, 3] when md.fermion."""
    gshape = tuple(op.dims[::-1]) + (4, 3, 3)
    for t, name in ((U, "U"), (P, "P")):
        if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous() and tuple(t.shape) == gshape):
            raise ValueError("%s must be a contiguous complex128 CUDA tensor of shape %s" % (name, gshape))
    if md.fermion:
        phi = _dev(phi, op.parity_shape, "phi")
    params = params or SolverParams(tol=1e-10, inner="f32", solver="cgne")
    cp = params.to_c()
    mp = md.to_c()
    st = _lib.MDStats()
    rc = load().lq_md_trajectory(op.handle, ctypes.byref(mp), ctypes.byref(cp), ctypes.c_void_p(U.data_ptr()),
                                 ctypes.c_void_p(P.data_ptr()),
                                 ctypes.c_void_p(phi.data_ptr()) if md.fermion else None, ctypes.byref(st), _stream())
    check(rc, allow_not_converged=True)
    return MDStats(st.H0, st.H1, st.dH, st.T0, st.T1, st.Sg0, st.Sg1, st.Sf0, st.Sf1, st.n_force, bool(st.converged),
                   st.iters, st.t_ms)


def hmc_step(op: Operator, U: torch.Tensor, P0: torch.Tensor, eta: torch.Tensor | None, r: float, md: MDParams,
             params: SolverParams | None = None):
    """One hybrid Monte Carlo update with the caller's random numbers: the
    momenta P0 (density exp(-1/2 tr P^dag P)), eta (pseudofermion heat bath
    phi = M^dag eta, density exp(-eta^dag eta)) and a uniform r in [0, 1).
    Returns (U_next, accepted, MDStats); U itself is not modified, and the
    operator holds U_next."""
    phi = None
    if md.fermion:
        op.set_gauge(U)
        phi = op.apply("schur_dag", eta, "f64")
    U1 = U.clone()
    P1 = P0.clone()
    st = md_trajectory(op, U1, P1, phi, md, params)
    accepted = bool(r < math.exp(min(0.0, -st.dH)))
    if not accepted:
        op.set_gauge(U)
        U1 = U
    return U1, accepted, st
