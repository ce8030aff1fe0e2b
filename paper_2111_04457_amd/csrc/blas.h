// blas.h -- vector kernels of the Krylov solvers on packed spinor fields.
//
// Solver scalars live in device memory, NSC doubles per system, so an
// iteration runs without host round trips: reduction kernels write
// per-workgroup partial sums (FP64) and a finish kernel sums them in a fixed
// order and performs the solver's scalar recurrence on the device.
// A field holding `sps` slices per system (1 for a parity field, 2 for a
// full field) is reduced over all slices of the system.
#pragma once

#include "fields.h"

namespace lq {

enum ScalarSlot {
    SC_RHO_RE = 0, SC_RHO_IM, SC_ALPHA_RE, SC_ALPHA_IM, SC_OMEGA_RE, SC_OMEGA_IM, SC_BETA_RE, SC_BETA_IM,
    SC_RR,       // current |r|^2 of the Krylov residual
    SC_TARGET2,  // stop when SC_RR <= SC_TARGET2 (set relative, made absolute by FIN_INIT_*)
    SC_DONE,     // 1: system converged (frozen)
    SC_BREAK,    // 1: breakdown (frozen, restart requested)
    SC_ITER,     // iterations performed
    SC_NORM2,    // result of FIN_NORM
    SC_SCALE,    // sqrt(SC_NORM2)
    SC_INVSCALE, // 1 / sqrt(SC_NORM2) (0 if zero)
    SC_ODONE,    // 1: outer residual already below target (inner solve skipped)
    SC_OTARGET2, // target of FIN_NORM for SC_ODONE
    SC_DOT_RE, SC_DOT_IM,
    SC_FORCE_BREAK,  // > 0: BiCGStab takes rho_new = 0 at this iteration (a breakdown forced from
                     // the host to exercise the restart path; 0 in every ordinary solve)
    SC_REINIT,       // reliable updates: 1 = the system starts a new Krylov space at the next
                     // restart (set by the host), 0 = it continues the one it has
    SC_RR_PREV,      // CG: |r|^2 of the iteration before the last one
    SC_RESCALE,      // reliable updates: |r| of the previous inner solve's source over the
                     // current one's (the factor between the two normalisations)
    NSC = 24
};
static_assert(SC_RESCALE < NSC, "solver scalar slots exceed NSC");

enum FinishOp {
    FIN_NORM = 0,       // K=1: SC_NORM2, SC_SCALE, SC_INVSCALE, SC_ODONE (vs SC_OTARGET2)
    FIN_INIT_CG,        // K=1: |r|^2 -> rr, done if rr <= target2 or outer done
    FIN_CG_ALPHA,       // K=1: |M p|^2 -> alpha = rr / |Mp|^2
    FIN_CG_BETA,        // K=1: |r|^2 -> beta, rr, iter, done
    FIN_INIT_BICG,      // K=1: |r|^2 -> rho = rr, alpha = omega = 1, done
    FIN_BICG_ALPHA,     // K=2: <rhat, v> -> alpha = rho / <rhat, v>
    FIN_BICG_OMEGA,     // K=3: <s, t>, |t|^2 -> omega = <t, s> / |t|^2
    FIN_BICG_RHO,       // K=3: <rhat, r>, |r|^2 -> beta, rho, rr, iter, done
    FIN_DOT,            // K=2: SC_DOT
    FIN_BICG_RESTART,   // K=3: <rhat, r>, |r|^2 of a replaced residual -> as FIN_INIT_BICG, but
                        // beta and rho continue the Krylov space (SC_REINIT = 0)
    FIN_CG_RESTART      // K=3: <p, r>, |r|^2 of a replaced residual -> as FIN_INIT_CG, and
                        // beta, omega for p = r + beta (p - omega r), which continues the
                        // search direction (SC_REINIT = 0)
};

// Per-slice reductions written to partial[(slice * nblocks + block) * K + k]
// (ragged fields: partial[tile * K + k]).  Every vector kernel also takes
// ragged fields (FieldView::tiles), all operands with the same slices.
enum ReduceMode { RED_NORM = 1, RED_DOT = 2, RED_DOT_NORM = 3 };

int blas_blocks(long n);

// partials of <x, y> / |x|^2 over every slice (y unused for RED_NORM);
// RED_DOT_NORM gives <x, y> and |y|^2.
// With mask (solver scalars, sps slices per system) frozen systems are
// skipped (their partials are zero).
hipError_t launch_reduce(FieldView x, FieldView y, int mode, double *partial, hipStream_t s,
                         const double *mask = nullptr, int sps = 1);
// finish: sums partials of nsys systems (sps slices each, nblocks per slice,
// K values; or, with range, range[sys].y partials from index range[sys].x:
// the partials of a ragged field's or a batched hop's systems) and runs op
// on the scalars sc[sys * NSC + ...].
hipError_t launch_finish(const double *partial, int nsys, int sps, int nblocks, int K, int op, double *sc,
                         double eps, hipStream_t s, const int2 *range = nullptr);

// Elementwise kernels (complex scalars read from sc of each slice's system,
// system = slice / sps; systems with SC_DONE or SC_BREAK set are skipped
// when skip_done is true).
hipError_t launch_zero(FieldView x, hipStream_t s);
// y = x converted to y's precision, times sc[SC_INVSCALE] if scaled
hipError_t launch_copy(FieldView y, FieldView x, const double *sc, int sps, bool scaled, hipStream_t s);
// x64 += sc[SC_SCALE] * e (scaled) or x64 += e
hipError_t launch_accum(FieldView x64, FieldView e, const double *sc, int sps, bool scaled, hipStream_t s);
// r = b - y and partial |r|^2
hipError_t launch_xmy_norm(FieldView r, FieldView b, FieldView y, double *partial, hipStream_t s);
// r64 -= sc[SC_SCALE] e (systems with SC_ODONE set keep r) and partial |r|^2
hipError_t launch_sub_scaled_norm(FieldView r64, FieldView e, const double *sc, int sps, double *partial,
                                  hipStream_t s);
// CG: x += alpha p; r -= alpha q; partial |r|^2
hipError_t launch_cg_xr(FieldView x, FieldView r, FieldView p, FieldView q, const double *sc, int sps,
                        double *partial, hipStream_t s);
// Reliable-update restarts: for the systems with SC_REINIT set (and the
// outer residual not yet converged) a = src, b = src (if b.base) and z = 0
// (if z.base); the other systems keep their vectors.
hipError_t launch_reinit(FieldView a, FieldView b, FieldView z, FieldView src, const double *sc, int sps,
                         hipStream_t s);
// CG: p = r + beta p (frozen systems keep p)
hipError_t launch_cg_p(FieldView p, FieldView r, const double *sc, int sps, hipStream_t s);
// BiCGStab: s = r - alpha v
hipError_t launch_bicg_s(FieldView sv, FieldView r, FieldView v, const double *sc, int sps, hipStream_t s);
// BiCGStab: x += alpha p + omega s; r = s - omega t; partials <rhat, r>, |r|^2
hipError_t launch_bicg_xr(FieldView x, FieldView r, FieldView p, FieldView sv, FieldView t, FieldView rhat,
                          const double *sc, int sps, double *partial, hipStream_t s);
// BiCGStab: p = r + beta (p - omega v)
hipError_t launch_bicg_p(FieldView p, FieldView r, FieldView v, const double *sc, int sps, hipStream_t s);
// apply gamma_5 = diag(1, 1, -1, -1) in place
hipError_t launch_gamma5(FieldView x, hipStream_t s);

}  // namespace lq
