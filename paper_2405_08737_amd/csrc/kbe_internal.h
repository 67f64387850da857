// Internal host-side interface between the C ABI layer and the kernel files of libkbe.
#pragma once

#include <hip/hip_runtime.h>

#include "kbe.h"

namespace kbe {

struct Params;

// Weights (kbe_weights.hip).
size_t weights_ws_bytes(int nt, int ntau);
hipError_t launch_weights(const kbe_grid *g, double *w, double *wtau, double *wf, void *ws,
                          hipStream_t st);
hipError_t launch_weights_dev(const double *t_d, const int32_t *o_d, int nt, int ntau,
                              double beta, int tau_order, double *w, double *wtau, double *wf,
                              void *ws, hipStream_t st);
hipError_t launch_grid_check(const double *t, const int32_t *order, int nt, int32_t *status,
                             hipStream_t st);
hipError_t launch_step_weights(const double *t, const int32_t *order, int nt, double *lam,
                               hipStream_t st);
hipError_t launch_interval_weights(double *t, int n, double tn, int kam, int kab, double *am,
                                   double *ab, hipStream_t st);

// Self-energy and its adjoint (kbe_sigma.hip).
hipError_t launch_sigma_row(const kbe_green *G, const double *u, int n, const kbe_sigma_row *out,
                            hipStream_t st);
hipError_t launch_add_blocks(const kbe_c128 *a, const kbe_c128 *b, kbe_c128 *out, int64_t cnt,
                             hipStream_t st);
hipError_t launch_sigma_batch(const kbe_sigma_batch_item *items_dev, int count, int64_t max_elems,
                              hipStream_t st);
hipError_t launch_sigma_full(const kbe_green *G, const double *u, const kbe_green *S,
                             hipStream_t st);
size_t sigma_vjp_ws_bytes(int N, int n, int ntau);
hipError_t launch_sigma_row_vjp(const kbe_green *G, const double *u, int n,
                                const kbe_sigma_row *gS, const kbe_green *gG, double *gu,
                                void *ws, hipStream_t st);

// Second-Born self-energy with a general four-index interaction (kbe_gf2.hip).
size_t gf2_ws_bytes(int N);
hipError_t launch_sigma_gf2(const kbe_green *G, const double *U, int n, const kbe_sigma_row *out,
                            void *ws, hipStream_t st);

// History integrals and their adjoint (kbe_collision.hip).
size_t collision_ws_bytes(int N, int nt, int ntau, int n, int m0, int m1, unsigned flags);
hipError_t launch_collision(const Params &p, unsigned flags, kbe_c128 *IR, kbe_c128 *IL,
                            kbe_c128 *Itv, kbe_c128 *Jtv, void *ws, hipStream_t st);
// Both forms of Eq. KBE2 in one call (the propagations): the lesser form's four outputs and the
// greater form's I^R, I^<, sharing the lesser form's I^R terms.  Internal flag (not part of the
// C ABI, whose flag check rejects it) for the workspace query and the task audit.
constexpr unsigned KBE_INT_BOTH = 0x10000u;
// Adjoint of the greater form's terms beyond the lesser form's (with KBE_GREATER; accumulate
// mode only): the G^R terms of I^R and the Sigma^R part of Sigma^> in I^<.  The adjoint of both
// forms is the lesser form's adjoint on the summed cotangents plus this on the greater form's.
constexpr unsigned KBE_INT_GREXTRA = 0x20000u;
// With KBE_INT_GREXTRA, set by the library when the cotangents of I^R and I^< are one array
// (the propagations): I^<'s Sigma^R terms and the G^R terms of I^R below the diagonal then share
// operand, streamed block and output, and run as one class.
constexpr unsigned KBE_INT_SAMECOT = 0x40000u;
hipError_t launch_collision_both(const Params &p, kbe_c128 *IRl, kbe_c128 *ILl, kbe_c128 *Itv,
                                 kbe_c128 *Jtv, kbe_c128 *IRg, kbe_c128 *ILg, void *ws,
                                 hipStream_t st);
size_t collision_vjp_ws_bytes(int N, int nt, int ntau, int n, int m0, int m1, unsigned flags);
// the largest workspace of a whole-row call at any n < nt (what a propagation reserves)
size_t collision_ws_bytes_rows(int N, int nt, int ntau, unsigned flags);
size_t collision_vjp_ws_bytes_rows(int N, int nt, int ntau, unsigned flags);
hipError_t launch_collision_vjp(const Params &p, unsigned flags, kbe_c128 *gmat,
                                const kbe_sigma_row *gS, void *ws, hipStream_t st);
// The lesser form's adjoint (p, flags; accumulate mode) and the greater form's extra terms on
// their own cotangents (pg, gflags = KBE_OUT_IR | KBE_OUT_IL | KBE_GREATER | KBE_INT_GREXTRA,
// gradients into gS and gSg), as two launch_collision_vjp calls would compute them; pg differs
// from p in its cotangents and flags only.  At 5 <= N <= 8 the Green's-function gradients of
// both take one pass.
hipError_t launch_collision_vjp_pair(const Params &p, unsigned flags, const Params &pg,
                                     unsigned gflags, kbe_c128 *gmat, const kbe_sigma_row *gS,
                                     const kbe_sigma_row *gSg, void *ws, hipStream_t st);

// Batches of history rows (kbe_batch.hip).
int batch_default_chunk();
size_t batch_ws_bytes(const kbe_batch_item *items, int count, int chunk);
hipError_t launch_batch(const kbe_batch_item *items, const kbe_batch_item *items_dev, int count,
                        int chunk, void *ws, hipStream_t st);
size_t batch_vjp_ws_bytes(int count);
hipError_t launch_batch_vjp(const kbe_batch_vjp_item *items_dev, int count, void *ws,
                            hipStream_t st);

// Fixed-grid propagation and its adjoint (kbe_prop.hip).
size_t prop_ws_bytes(int N, int nt, int ntau, int64_t ldt, int K);
hipError_t launch_propagate(const kbe_prop *P, const kbe_wts *W, const kbe_green *G,
                            double *dens, void *ws, hipStream_t st);
hipError_t launch_propagate_vjp(const kbe_prop *P, const kbe_wts *W, const kbe_green *G,
                                const double *gdens, double *gu, double *gamp, void *ws,
                                hipStream_t st);
size_t equilibrium_ws_bytes(int N, int ntau);
hipError_t launch_equilibrium(int N, int ntau, double beta, const double *wf, const double *h0,
                              const double *u, double mu, double mix, double tol, int maxit,
                              kbe_c128 *mat, void *ws, hipStream_t st, int *iterations,
                              double *change);
size_t prop_adaptive_ws_bytes(int N, int nt, int ntau);
hipError_t launch_propagate_adaptive(const kbe_prop *P, const kbe_adapt_ctl *ctl,
                                     const kbe_wts *W, const kbe_green *G, double *dens,
                                     kbe_adapt_trace *tr, void *ws, hipStream_t st,
                                     int *stalled);

}  // namespace kbe

// Host-side self-check of the collision kernels' work decomposition (no GPU needed): for the
// plan kbe_collision (adjoint = 0) or kbe_collision_vjp (adjoint = 1) would launch with these
// sizes and flags, walks every task as the kernels do and returns how many of the addresses they
// form (staged operand blocks over the workgroup's union of term ranges, weights and streamed
// blocks of each output's own terms) fall outside their arrays; *terms_checked receives the
// number of addresses examined.  Not part of the public ABI (used by the test-suite).
extern "C" int64_t kbe_internal_audit_tasks(int32_t N, int32_t nt, int32_t ntau, int64_t ldt,
                                            int32_t n, int32_t m0, int32_t m1, uint32_t flags,
                                            int32_t adjoint, int64_t *terms_checked);

// Ceiling microbenchmarks (kbe_ceilings.hip; used by the benchmark's --ceilings mode).
// kind 0: FP64 MFMA 4x4x4 stream, 1: FP64 MFMA 16x16x4 stream, 2: HBM read of `bytes` from src,
// 3: copy of `bytes` from src to dst.  out: device doubles, kbe_internal_ceiling_out_count() of
// them.  Returns 0, or 1 for a bad kind, 4 for a launch failure.
extern "C" int32_t kbe_internal_ceiling_run(int32_t kind, const void *src, void *dst,
                                            int64_t bytes, double *out, int32_t iters,
                                            void *stream);
// FLOP (kinds 0, 1) or HBM bytes (kinds 2, 3) of one launch.
extern "C" double kbe_internal_ceiling_counts(int32_t kind, int64_t bytes, int32_t iters);
extern "C" int64_t kbe_internal_ceiling_out_count(void);

