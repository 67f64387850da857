// C ABI of libkbe: argument validation (before anything is enqueued), dispatch to the kernel
// files, status codes and the thread-local error text.  See include/kbe.h for the contract.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "kbe_dev.h"
#include "kbe_internal.h"

namespace {

thread_local std::string g_err;

kbe_status fail(kbe_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

kbe_status ok() {
  g_err.clear();
  return KBE_OK;
}

kbe_status hip_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return ok();
  return fail(KBE_EHIP, "%s: %s", what, hipGetErrorString(e));
}

kbe_status check_green(const kbe_green *G, const char *name) {
  if (!G) return fail(KBE_EINVAL, "%s is NULL", name);
  if (G->N < 1 || G->N > KBE_NMAX) return fail(KBE_EINVAL, "%s->N = %d outside 1..%d", name, G->N, KBE_NMAX);
  if (G->nt < 1) return fail(KBE_EINVAL, "%s->nt = %d < 1", name, G->nt);
  if (G->ntau < 0 || G->ntau == 1) return fail(KBE_EINVAL, "%s->ntau = %d (must be 0 or >= 2)", name, G->ntau);
  if (G->ldt < G->nt) return fail(KBE_EINVAL, "%s->ldt = %lld < nt = %d", name, (long long)G->ldt, G->nt);
  if (!G->kp || !G->rdiag) return fail(KBE_EINVAL, "%s->kp or %s->rdiag is NULL", name, name);
  if (G->ntau > 0 && (!G->tv || !G->mat)) return fail(KBE_EINVAL, "%s->tv or %s->mat is NULL with ntau > 0", name, name);
  return KBE_OK;
}

kbe_status check_same_shape(const kbe_green *G, const kbe_green *H, const char *name) {
  kbe_status s = check_green(H, name);
  if (s != KBE_OK) return s;
  if (H->N != G->N || H->nt != G->nt || H->ntau != G->ntau || H->ldt != G->ldt)
    return fail(KBE_EINVAL, "%s does not have the shape of G", name);
  return KBE_OK;
}

kbe_status check_common(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W, int n,
                        int m0, int m1, unsigned flags) {
  kbe_status s = check_green(G, "G");
  if (s != KBE_OK) return s;
  if (flags & ~(KBE_OUT_ALL | KBE_FORCE_GENERIC | KBE_GRAD_OVERWRITE | KBE_GREATER))
    return fail(KBE_EINVAL, "unknown flag bits 0x%x", flags);
  if (n < 0 || n >= G->nt) return fail(KBE_ERANGE, "n = %d outside [0, nt = %d)", n, G->nt);
  if (m0 < 0 || m0 > m1 || m1 > n + 1)
    return fail(KBE_ERANGE, "m-range [%d, %d) not inside [0, n+1 = %d]", m0, m1, n + 1);
  if (!S) return fail(KBE_EINVAL, "S is NULL");
  if (!W) return fail(KBE_EINVAL, "W is NULL");
  const bool th = G->ntau > 0;
  const unsigned need_ret = KBE_OUT_IR | KBE_OUT_JTV | ((flags & KBE_GREATER) ? KBE_OUT_IL : 0u);
  if ((flags & need_ret) && !S->ret) return fail(KBE_EINVAL, "S->ret is NULL");
  if ((flags & KBE_OUT_IL) && !S->les) return fail(KBE_EINVAL, "S->les is NULL");
  if (th && (flags & (KBE_OUT_ITV | KBE_OUT_JTV)) && !S->tv) return fail(KBE_EINVAL, "S->tv is NULL");
  if ((flags & (KBE_OUT_IR | KBE_OUT_IL | KBE_OUT_JTV)) && !W->w) return fail(KBE_EINVAL, "W->w is NULL");
  if (th && (flags & KBE_OUT_ITV) && !W->wtau) return fail(KBE_EINVAL, "W->wtau is NULL");
  if (th && (flags & KBE_OUT_JTV) && !W->wtau_fwd) return fail(KBE_EINVAL, "W->wtau_fwd is NULL");
  return KBE_OK;
}

kbe::Params make_params(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W, int n,
                        int m0, int m1, unsigned flags) {
  kbe::Params p{};
  p.N = G->N;
  p.nt = G->nt;
  p.ntau = G->ntau;
  p.J = G->ntau - 1;
  p.n = n;
  p.m0 = m0;
  p.m1 = m1;
  p.ldt = G->ldt;
  p.kp = G->kp;
  p.rdiag = G->rdiag;
  p.tv = G->tv;
  p.mat = G->mat;
  p.ret = S->ret;
  p.les = S->les;
  p.stv = S->tv;
  p.w = W->w;
  p.wtau = W->wtau;
  p.wf = W->wtau_fwd;
  p.fIR = (flags & KBE_OUT_IR) != 0;
  p.fIL = (flags & KBE_OUT_IL) != 0;
  p.fITV = (flags & KBE_OUT_ITV) && G->ntau > 0;
  p.fJTV = (flags & KBE_OUT_JTV) && G->ntau > 0;
  p.overwrite = (flags & KBE_GRAD_OVERWRITE) != 0;
  return p;
}

}  // namespace

extern "C" {

const char *kbe_status_string(kbe_status s) {
  switch (s) {
    case KBE_OK: return "KBE_OK";
    case KBE_EINVAL: return "KBE_EINVAL: invalid argument";
    case KBE_ERANGE: return "KBE_ERANGE: index or order out of range";
    case KBE_ENOMEM: return "KBE_ENOMEM: workspace too small";
    case KBE_EHIP: return "KBE_EHIP: HIP runtime error";
    case KBE_ENOTSUP: return "KBE_ENOTSUP: not supported";
    case KBE_ESTEP: return "KBE_ESTEP: adaptive controller stopped before t_end";
    case KBE_ECONV: return "KBE_ECONV: equilibrium iteration did not converge";
  }
  return "unknown kbe_status";
}

const char *kbe_last_error(void) { return g_err.c_str(); }

int32_t kbe_version(void) { return 10000; }

size_t kbe_weights_workspace(const kbe_grid *g) {
  if (!g || g->nt < 1) return 0;
  return kbe::weights_ws_bytes(g->nt, g->ntau > 0 ? g->ntau : 0);
}

kbe_status kbe_weights(const kbe_grid *g, double *w, double *wtau, double *wtau_fwd, void *ws,
                       size_t ws_bytes, void *stream) {
  if (!g) return fail(KBE_EINVAL, "grid is NULL");
  if (g->nt < 1) return fail(KBE_EINVAL, "nt = %d < 1", g->nt);
  if (!g->t || !g->order) return fail(KBE_EINVAL, "grid t or order is NULL");
  if (!w) return fail(KBE_EINVAL, "w is NULL");
  if (g->t[0] != 0.0) return fail(KBE_EINVAL, "t[0] = %g, the grid must start at 0", g->t[0]);
  for (int p = 1; p < g->nt; ++p) {
    if (!(g->t[p] > g->t[p - 1]) || !std::isfinite(g->t[p]))
      return fail(KBE_EINVAL, "t is not strictly increasing at p = %d", p);
    if (g->order[p] < 1 || g->order[p] > KBE_KMAX)
      return fail(KBE_ERANGE, "order[%d] = %d outside 1..%d", p, g->order[p], KBE_KMAX);
  }
  if (g->ntau < 0 || g->ntau == 1) return fail(KBE_EINVAL, "ntau = %d (must be 0 or >= 2)", g->ntau);
  if (g->ntau > 0) {
    if (!(g->beta > 0.0) || !std::isfinite(g->beta)) return fail(KBE_EINVAL, "beta = %g must be > 0", g->beta);
    if (g->tau_order < 1 || g->tau_order > KBE_KMAX)
      return fail(KBE_ERANGE, "tau_order = %d outside 1..%d", g->tau_order, KBE_KMAX);
    if (!wtau || !wtau_fwd) return fail(KBE_EINVAL, "wtau or wtau_fwd is NULL with ntau > 0");
  }
  const size_t need = kbe_weights_workspace(g);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing((hipStream_t)stream, &cap);
  if (e != hipSuccess) return hip_status(e, "kbe_weights");
  if (cap != hipStreamCaptureStatusNone)
    return fail(KBE_ENOTSUP, "kbe_weights copies host memory and cannot be captured: use "
                             "kbe_weights_dev");
  e = kbe::launch_weights(g, w, wtau, wtau_fwd, ws, (hipStream_t)stream);
  return hip_status(e, "kbe_weights");
}

kbe_status kbe_sigma_2b(const kbe_green *G, const double *u, int32_t n, const kbe_sigma_row *out,
                        void *stream) {
  kbe_status s = check_green(G, "G");
  if (s != KBE_OK) return s;
  if (n < 0 || n >= G->nt) return fail(KBE_ERANGE, "n = %d outside [0, nt = %d)", n, G->nt);
  if (!u) return fail(KBE_EINVAL, "u is NULL");
  if (!out || !out->ret || !out->les) return fail(KBE_EINVAL, "output row is NULL");
  if (G->ntau > 0 && !out->tv) return fail(KBE_EINVAL, "out->tv is NULL with ntau > 0");
  return hip_status(kbe::launch_sigma_row(G, u, n, out, (hipStream_t)stream), "kbe_sigma_2b");
}

kbe_status kbe_sigma_2b_full(const kbe_green *G, const double *u, const kbe_green *S,
                             void *stream) {
  kbe_status s = check_green(G, "G");
  if (s != KBE_OK) return s;
  if (!u) return fail(KBE_EINVAL, "u is NULL");
  if (!S || !S->kp || !S->rdiag) return fail(KBE_EINVAL, "S, S->kp or S->rdiag is NULL");
  if (S->N != G->N || S->nt != G->nt || S->ntau != G->ntau || S->ldt < S->nt)
    return fail(KBE_EINVAL, "S shape (N %d, nt %d, ntau %d, ldt %lld) does not match G", S->N,
                S->nt, S->ntau, (long long)S->ldt);
  if (G->ntau > 0 && !S->tv) return fail(KBE_EINVAL, "S->tv is NULL with ntau > 0");
  return hip_status(kbe::launch_sigma_full(G, u, S, (hipStream_t)stream), "kbe_sigma_2b_full");
}

kbe_status kbe_sigma_2b_batch(const kbe_sigma_batch_item *items,
                              const kbe_sigma_batch_item *items_dev, int32_t count, void *stream) {
  if (count < 0 || count > KBE_BATCH_MAX)
    return fail(KBE_ERANGE, "count = %d outside [0, %d]", count, KBE_BATCH_MAX);
  if (count == 0) return ok();
  if (!items || !items_dev) return fail(KBE_EINVAL, "items or items_dev is NULL");
  int64_t max_elems = 0;
  for (int32_t i = 0; i < count; ++i) {
    const kbe_sigma_batch_item &it = items[i];
    if (it.N < 1 || it.N > KBE_NMAX)
      return fail(KBE_EINVAL, "item %d: N = %d outside 1..%d", i, it.N, KBE_NMAX);
    if (it.nt < 1) return fail(KBE_EINVAL, "item %d: nt = %d < 1", i, it.nt);
    if (it.ntau < 0 || it.ntau == 1)
      return fail(KBE_EINVAL, "item %d: ntau = %d (must be 0 or >= 2)", i, it.ntau);
    if (it.ldt < it.nt)
      return fail(KBE_EINVAL, "item %d: ldt = %lld < nt = %d", i, (long long)it.ldt, it.nt);
    if (it.n < 0 || it.n >= it.nt)
      return fail(KBE_ERANGE, "item %d: n = %d outside [0, nt = %d)", i, it.n, it.nt);
    if (!it.kp || !it.rdiag || !it.u || !it.ret || !it.les)
      return fail(KBE_EINVAL, "item %d: kp, rdiag, u, ret or les is NULL", i);
    if (it.ntau > 0 && (!it.tv || !it.stv))
      return fail(KBE_EINVAL, "item %d: tv or stv is NULL with ntau > 0", i);
    const int64_t e = (int64_t)(it.n + 1 + it.ntau) * it.N * it.N;
    max_elems = e > max_elems ? e : max_elems;
  }
  return hip_status(kbe::launch_sigma_batch(items_dev, count, max_elems, (hipStream_t)stream),
                    "kbe_sigma_2b_batch");
}

size_t kbe_sigma_gf2_workspace(int32_t N) {
  if (N < 1 || N > KBE_NMAX) return 0;
  return kbe::gf2_ws_bytes(N);
}

kbe_status kbe_sigma_gf2(const kbe_green *G, const double *U, int32_t n, const kbe_sigma_row *out,
                         void *ws, size_t ws_bytes, void *stream) {
  kbe_status s = check_green(G, "G");
  if (s != KBE_OK) return s;
  if (n < 0 || n >= G->nt) return fail(KBE_ERANGE, "n = %d outside [0, nt = %d)", n, G->nt);
  if (!U) return fail(KBE_EINVAL, "U is NULL");
  if (!out || !out->ret || !out->les) return fail(KBE_EINVAL, "output row is NULL");
  if (G->ntau > 0 && !out->tv) return fail(KBE_EINVAL, "out->tv is NULL with ntau > 0");
  const size_t need = kbe::gf2_ws_bytes(G->N);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  return hip_status(kbe::launch_sigma_gf2(G, U, n, out, ws, (hipStream_t)stream), "kbe_sigma_gf2");
}

size_t kbe_sigma_2b_vjp_workspace(int32_t N, int32_t n, int32_t ntau) {
  if (N < 1 || n < 0 || ntau < 0) return 0;
  return kbe::sigma_vjp_ws_bytes(N, n, ntau);
}

kbe_status kbe_sigma_2b_vjp(const kbe_green *G, const double *u, int32_t n,
                            const kbe_sigma_row *gS, const kbe_green *gG, double *gu, void *ws,
                            size_t ws_bytes, void *stream) {
  kbe_status s = check_green(G, "G");
  if (s != KBE_OK) return s;
  if ((s = check_same_shape(G, gG, "gG")) != KBE_OK) return s;
  if (n < 0 || n >= G->nt) return fail(KBE_ERANGE, "n = %d outside [0, nt = %d)", n, G->nt);
  if (!u || !gu) return fail(KBE_EINVAL, "u or gu is NULL");
  if (!gS || !gS->ret || !gS->les) return fail(KBE_EINVAL, "gS row is NULL");
  if (G->ntau > 0 && !gS->tv) return fail(KBE_EINVAL, "gS->tv is NULL with ntau > 0");
  const size_t need = kbe_sigma_2b_vjp_workspace(G->N, n, G->ntau);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  return hip_status(kbe::launch_sigma_row_vjp(G, u, n, gS, gG, gu, ws, (hipStream_t)stream),
                    "kbe_sigma_2b_vjp");
}

size_t kbe_collision_workspace(int32_t N, int32_t nt, int32_t ntau, int32_t n, int32_t m0,
                               int32_t m1, uint32_t flags) {
  if (N < 1 || N > KBE_NMAX || n < 0 || m0 < 0 || m1 < m0 || ntau < 0) return 0;
  return kbe::collision_ws_bytes(N, nt, ntau, n, m0, m1, flags);
}

kbe_status kbe_collision(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W, int32_t n,
                         int32_t m0, int32_t m1, uint32_t flags, kbe_c128 *IR, kbe_c128 *IL,
                         kbe_c128 *Itv, kbe_c128 *Jtv, void *ws, size_t ws_bytes, void *stream) {
  kbe_status s = check_common(G, S, W, n, m0, m1, flags);
  if (s != KBE_OK) return s;
  const bool M = m1 > m0;
  if ((flags & KBE_OUT_IR) && M && !IR) return fail(KBE_EINVAL, "IR is NULL");
  if ((flags & KBE_OUT_IL) && M && !IL) return fail(KBE_EINVAL, "IL is NULL");
  if ((flags & KBE_OUT_ITV) && M && !Itv) return fail(KBE_EINVAL, "Itv is NULL");
  if ((flags & KBE_OUT_JTV) && G->ntau > 0 && !Jtv) return fail(KBE_EINVAL, "Jtv is NULL");
  const size_t need = kbe_collision_workspace(G->N, G->nt, G->ntau, n, m0, m1, flags);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  kbe::Params p = make_params(G, S, W, n, m0, m1, flags);
  return hip_status(kbe::launch_collision(p, flags, IR, IL, Itv, Jtv, ws, (hipStream_t)stream),
                    "kbe_collision");
}

size_t kbe_collision_both_workspace(int32_t N, int32_t nt, int32_t ntau, int32_t n, int32_t m0,
                                    int32_t m1) {
  if (N < 1 || N > KBE_NMAX || n < 0 || m0 < 0 || m1 < m0 || ntau < 0) return 0;
  return kbe::collision_ws_bytes(N, nt, ntau, n, m0, m1, KBE_OUT_ALL | kbe::KBE_INT_BOTH);
}

kbe_status kbe_collision_both(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W,
                              int32_t n, int32_t m0, int32_t m1, kbe_c128 *IR, kbe_c128 *IL,
                              kbe_c128 *Itv, kbe_c128 *Jtv, kbe_c128 *IRg, kbe_c128 *ILg,
                              void *ws, size_t ws_bytes, void *stream) {
  kbe_status s = check_common(G, S, W, n, m0, m1, KBE_OUT_ALL | KBE_GREATER);
  if (s != KBE_OK) return s;
  const bool M = m1 > m0, th = G->ntau > 0;
  if (M && (!IR || !IL || !IRg || !ILg)) return fail(KBE_EINVAL, "IR, IL, IRg or ILg is NULL");
  if (M && th && !Itv) return fail(KBE_EINVAL, "Itv is NULL");
  if (th && !Jtv) return fail(KBE_EINVAL, "Jtv is NULL");
  const size_t need = kbe_collision_both_workspace(G->N, G->nt, G->ntau, n, m0, m1);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  kbe::Params p = make_params(G, S, W, n, m0, m1, KBE_OUT_ALL);
  return hip_status(kbe::launch_collision_both(p, IR, IL, th ? Itv : nullptr, th ? Jtv : nullptr,
                                               IRg, ILg, ws, (hipStream_t)stream),
                    "kbe_collision_both");
}

// ---------------------------------------------------------------------------------------
// kbe_collision_noalloc: kbe_collision with its workspace in a fixed device array.
//
// `scratch` is the array; each device the library runs on holds its own copy from the time
// the library's code object is loaded there until the process ends.  In host code the name is
// only a host-side stand-in: the device address comes from hipGetSymbolAddress, taken once per
// device with that device current and kept in g_scratch_dev, and only that address is handed to
// the kernels.
// ---------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[KBE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];

// Device address of `scratch` on the device that owns `stream` (the current device for the
// NULL stream).
kbe_status scratch_address(hipStream_t stream, void **out) {
  int cur = 0, dev = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_status(e, "hipGetDevice");
  dev = cur;
  if (stream) {
    e = hipStreamGetDevice(stream, &dev);
    if (e != hipSuccess) return hip_status(e, "hipStreamGetDevice");
  }
  if (dev < 0 || dev >= kMaxDevices) return fail(KBE_ENOTSUP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return hip_status(e, "hipSetDevice");
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    const hipError_t r = dev != cur ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
    if (r != hipSuccess) return hip_status(r, "hipSetDevice");
    if (!ptr) return fail(KBE_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return KBE_OK;
}
}  // namespace

kbe_status kbe_collision_noalloc(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W,
                                 int32_t n, int32_t m0, int32_t m1, uint32_t flags, kbe_c128 *IR,
                                 kbe_c128 *IL, kbe_c128 *Itv, kbe_c128 *Jtv, void *stream) {
  kbe_status s = check_common(G, S, W, n, m0, m1, flags);
  if (s != KBE_OK) return s;
  const bool M = m1 > m0;
  if ((flags & KBE_OUT_IR) && M && !IR) return fail(KBE_EINVAL, "IR is NULL");
  if ((flags & KBE_OUT_IL) && M && !IL) return fail(KBE_EINVAL, "IL is NULL");
  if ((flags & KBE_OUT_ITV) && M && !Itv) return fail(KBE_EINVAL, "Itv is NULL");
  if ((flags & KBE_OUT_JTV) && G->ntau > 0 && !Jtv) return fail(KBE_EINVAL, "Jtv is NULL");
  const size_t need = kbe_collision_workspace(G->N, G->nt, G->ntau, n, m0, m1, flags);
  if (need > (size_t)KBE_NOALLOC_SCRATCH_BYTES)
    return fail(KBE_ENOMEM, "this call needs %zu bytes of scratch, more than the fixed %zu",
                need, (size_t)KBE_NOALLOC_SCRATCH_BYTES);
  void *ws = nullptr;
  if ((s = scratch_address((hipStream_t)stream, &ws)) != KBE_OK) return s;
  kbe::Params p = make_params(G, S, W, n, m0, m1, flags);
  return hip_status(kbe::launch_collision(p, flags, IR, IL, Itv, Jtv, ws, (hipStream_t)stream),
                    "kbe_collision_noalloc");
}

size_t kbe_collision_vjp_workspace(int32_t N, int32_t nt, int32_t ntau, int32_t n, int32_t m0,
                                   int32_t m1, uint32_t flags) {
  if (N < 1 || N > KBE_NMAX || n < 0 || m0 < 0 || m1 < m0 || ntau < 0) return 0;
  return kbe::collision_vjp_ws_bytes(N, nt, ntau, n, m0, m1, flags);
}

kbe_status kbe_collision_vjp(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W,
                             int32_t n, int32_t m0, int32_t m1, uint32_t flags,
                             const kbe_c128 *gIR, const kbe_c128 *gIL, const kbe_c128 *gItv,
                             const kbe_c128 *gJtv, const kbe_green *gG, const kbe_sigma_row *gS,
                             void *ws, size_t ws_bytes, void *stream) {
  kbe_status s = check_common(G, S, W, n, m0, m1, flags);
  if (s != KBE_OK) return s;
  if ((s = check_same_shape(G, gG, "gG")) != KBE_OK) return s;
  const bool M = m1 > m0, th = G->ntau > 0;
  if ((flags & KBE_OUT_IR) && M && !gIR) return fail(KBE_EINVAL, "gIR is NULL");
  if ((flags & KBE_OUT_IL) && M && !gIL) return fail(KBE_EINVAL, "gIL is NULL");
  if ((flags & KBE_OUT_ITV) && M && th && !gItv) return fail(KBE_EINVAL, "gItv is NULL");
  if ((flags & KBE_OUT_JTV) && th && !gJtv) return fail(KBE_EINVAL, "gJtv is NULL");
  if ((flags & KBE_OUT_IR) && !S->ret) return fail(KBE_EINVAL, "S->ret is NULL");
  if (!gS || !gS->ret || !gS->les) return fail(KBE_EINVAL, "gS row is NULL");
  if (th && !gS->tv) return fail(KBE_EINVAL, "gS->tv is NULL with ntau > 0");
  const size_t need = kbe_collision_vjp_workspace(G->N, G->nt, G->ntau, n, m0, m1, flags);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  kbe::Params p = make_params(G, S, W, n, m0, m1, flags);
  p.gIR = gIR;
  p.gIL = gIL;
  p.gItv = gItv;
  p.gJ = gJtv;
  p.gkp = gG->kp;
  p.grdiag = gG->rdiag;
  p.gtv = gG->tv;
  return hip_status(kbe::launch_collision_vjp(p, flags, gG->mat, gS, ws, (hipStream_t)stream),
                    "kbe_collision_vjp");
}

// ---------------------------------------------------------------------------------------
// Adjoint of both forms: the lesser adjoint on the summed cotangents, then the greater form's
// own terms.  Workspace: [collision adjoint][gIR + gIRg][gIL + gILg][the second pass's gS].
// ---------------------------------------------------------------------------------------
namespace {
constexpr unsigned FG_EXTRA = KBE_OUT_IR | KBE_OUT_IL | KBE_GREATER | kbe::KBE_INT_GREXTRA;

size_t al256c(size_t x) { return (x + 255) & ~(size_t)255; }

size_t both_vjp_layout(int N, int nt, int ntau, int n, int m0, int m1, size_t off[5]) {
  const size_t E = (size_t)N * N * sizeof(kbe_c128);
  const size_t a = kbe::collision_vjp_ws_bytes(N, nt, ntau, n, m0, m1, KBE_OUT_ALL);
  const size_t b = kbe::collision_vjp_ws_bytes(N, nt, ntau, n, m0, m1, FG_EXTRA);
  size_t t = al256c(a > b ? a : b);
  off[0] = t;  // gIR + gIRg
  t += al256c((size_t)(m1 - m0) * E);
  off[1] = t;  // gIL + gILg
  t += al256c((size_t)(m1 - m0) * E);
  off[2] = t;  // second pass: gS ret
  t += al256c((size_t)(n + 1) * E);
  off[3] = t;  // les
  t += al256c((size_t)(n + 1) * E);
  off[4] = t;  // tv
  t += al256c((size_t)(ntau > 0 ? ntau : 1) * E);
  return t;
}
}  // namespace

size_t kbe_collision_both_vjp_workspace(int32_t N, int32_t nt, int32_t ntau, int32_t n,
                                        int32_t m0, int32_t m1) {
  if (N < 1 || N > KBE_NMAX || n < 0 || m0 < 0 || m1 < m0 || ntau < 0) return 0;
  size_t off[5];
  return both_vjp_layout(N, nt, ntau, n, m0, m1, off);
}

kbe_status kbe_collision_both_vjp(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W,
                                  int32_t n, int32_t m0, int32_t m1, const kbe_c128 *gIR,
                                  const kbe_c128 *gIL, const kbe_c128 *gItv,
                                  const kbe_c128 *gJtv, const kbe_c128 *gIRg,
                                  const kbe_c128 *gILg, const kbe_green *gG,
                                  const kbe_sigma_row *gS, void *ws, size_t ws_bytes,
                                  void *stream) {
  kbe_status s = check_common(G, S, W, n, m0, m1, KBE_OUT_ALL | KBE_GREATER);
  if (s != KBE_OK) return s;
  if ((s = check_same_shape(G, gG, "gG")) != KBE_OK) return s;
  const bool M = m1 > m0, th = G->ntau > 0;
  if (M && (!gIR || !gIL || !gIRg || !gILg))
    return fail(KBE_EINVAL, "gIR, gIL, gIRg or gILg is NULL");
  if (M && th && !gItv) return fail(KBE_EINVAL, "gItv is NULL");
  if (th && !gJtv) return fail(KBE_EINVAL, "gJtv is NULL");
  if (!gS || !gS->ret || !gS->les) return fail(KBE_EINVAL, "gS row is NULL");
  if (th && !gS->tv) return fail(KBE_EINVAL, "gS->tv is NULL with ntau > 0");
  size_t off[5];
  const size_t need = both_vjp_layout(G->N, G->nt, G->ntau, n, m0, m1, off);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  const hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  const int64_t E = (int64_t)G->N * G->N, cnt = (int64_t)(m1 - m0) * E;
  kbe_c128 *cIR = (kbe_c128 *)(w + off[0]), *cIL = (kbe_c128 *)(w + off[1]);
  hipError_t e = kbe::launch_add_blocks(gIR, gIRg, cIR, M ? cnt : 0, st);
  if (e == hipSuccess) e = kbe::launch_add_blocks(gIL, gILg, cIL, M ? cnt : 0, st);
  if ((s = hip_status(e, "kbe_collision_both_vjp")) != KBE_OK) return s;
  kbe::Params p = make_params(G, S, W, n, m0, m1, KBE_OUT_ALL);
  p.gIR = cIR;
  p.gIL = cIL;
  p.gItv = gItv;
  p.gJ = gJtv;
  p.gkp = gG->kp;
  p.grdiag = gG->rdiag;
  p.gtv = gG->tv;
  kbe::Params q = make_params(G, S, W, n, m0, m1, FG_EXTRA);
  q.gIR = gIRg;
  q.gIL = gILg;
  q.gkp = gG->kp;
  q.grdiag = gG->rdiag;
  q.gtv = gG->tv;
  kbe_sigma_row g2{(kbe_c128 *)(w + off[2]), (kbe_c128 *)(w + off[3]),
                   th ? (kbe_c128 *)(w + off[4]) : nullptr};
  s = hip_status(kbe::launch_collision_vjp_pair(p, KBE_OUT_ALL, q, FG_EXTRA, gG->mat, gS, &g2,
                                                ws, st),
                 "kbe_collision_both_vjp");
  if (s != KBE_OK) return s;
  const int64_t rows = (int64_t)(n + 1) * E;
  e = kbe::launch_add_blocks(gS->ret, g2.ret, gS->ret, rows, st);
  if (e == hipSuccess) e = kbe::launch_add_blocks(gS->les, g2.les, gS->les, rows, st);
  return hip_status(e, "kbe_collision_both_vjp");
}

// ---------------------------------------------------------------------------------------
// Weights from a device-resident grid; step weights; the fixed-grid propagation.
// ---------------------------------------------------------------------------------------
size_t kbe_weights_dev_workspace(int32_t nt, int32_t ntau) {
  if (nt < 1 || ntau < 0) return 0;
  return kbe::weights_ws_bytes(nt, ntau);
}

kbe_status kbe_weights_dev(const double *t, const int32_t *order, int32_t nt, int32_t ntau,
                           double beta, int32_t tau_order, double *w, double *wtau,
                           double *wtau_fwd, int32_t *status, void *ws, size_t ws_bytes,
                           void *stream) {
  if (!t || !order || !w) return fail(KBE_EINVAL, "t, order or w is NULL");
  if (nt < 1) return fail(KBE_EINVAL, "nt = %d < 1", nt);
  if (ntau < 0 || ntau == 1) return fail(KBE_EINVAL, "ntau = %d (must be 0 or >= 2)", ntau);
  if (ntau > 0) {
    if (!(beta > 0)) return fail(KBE_EINVAL, "beta = %g <= 0", beta);
    if (tau_order < 1 || tau_order > KBE_KMAX)
      return fail(KBE_ERANGE, "tau_order = %d outside 1..%d", tau_order, KBE_KMAX);
    if (!wtau || !wtau_fwd) return fail(KBE_EINVAL, "wtau or wtau_fwd is NULL with ntau > 0");
  }
  const size_t need = kbe_weights_dev_workspace(nt, ntau);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  if (status) {
    hipError_t e = kbe::launch_grid_check(t, order, nt, status, st);
    if (e != hipSuccess) return hip_status(e, "kbe_weights_dev");
  }
  return hip_status(kbe::launch_weights_dev(t, order, nt, ntau, beta, tau_order, w, wtau,
                                            wtau_fwd, ws, st),
                    "kbe_weights_dev");
}

kbe_status kbe_step_weights(const double *t, const int32_t *order, int32_t nt, double *lam,
                            int32_t *status, void *stream) {
  if (!t || !order || !lam) return fail(KBE_EINVAL, "t, order or lam is NULL");
  if (nt < 1) return fail(KBE_EINVAL, "nt = %d < 1", nt);
  hipStream_t st = (hipStream_t)stream;
  if (status) {
    hipError_t e = kbe::launch_grid_check(t, order, nt, status, st);
    if (e != hipSuccess) return hip_status(e, "kbe_step_weights");
  }
  return hip_status(kbe::launch_step_weights(t, order, nt, lam, st), "kbe_step_weights");
}

size_t kbe_propagate_workspace(int32_t N, int32_t nt, int32_t ntau, int64_t ldt, int32_t iters) {
  if (N < 1 || N > KBE_NMAX || nt < 1 || ntau < 0 || ntau == 1 || ldt < nt || iters < 1) return 0;
  return kbe::prop_ws_bytes(N, nt, ntau, ldt, iters);
}

namespace {
kbe_status check_prop(const kbe_prop *P, const kbe_wts *W, const kbe_green *G, size_t ws_bytes,
                      const void *ws) {
  kbe_status s = check_green(G, "G");
  if (s != KBE_OK) return s;
  if (!P || !W) return fail(KBE_EINVAL, "P or W is NULL");
  if (P->iters < 1) return fail(KBE_EINVAL, "iters = %d < 1", P->iters);
  if (!P->h0 || !P->u || !P->t || !P->order || !P->lam)
    return fail(KBE_EINVAL, "P->h0, u, t, order or lam is NULL");
  if (!(P->pulse_sigma > 0)) return fail(KBE_EINVAL, "pulse_sigma = %g <= 0", P->pulse_sigma);
  if (!W->w) return fail(KBE_EINVAL, "W->w is NULL");
  if (G->ntau > 0 && (!W->wtau || !W->wtau_fwd))
    return fail(KBE_EINVAL, "tau weights are NULL with ntau > 0");
  const size_t need = kbe_propagate_workspace(G->N, G->nt, G->ntau, G->ldt, P->iters);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  return KBE_OK;
}
}  // namespace

kbe_status kbe_propagate(const kbe_prop *P, const kbe_wts *W, const kbe_green *G, double *dens,
                         void *ws, size_t ws_bytes, void *stream) {
  kbe_status s = check_prop(P, W, G, ws_bytes, ws);
  if (s != KBE_OK) return s;
  if (!dens) return fail(KBE_EINVAL, "dens is NULL");
  return hip_status(kbe::launch_propagate(P, W, G, dens, ws, (hipStream_t)stream),
                    "kbe_propagate");
}

kbe_status kbe_propagate_vjp(const kbe_prop *P, const kbe_wts *W, const kbe_green *G,
                             const double *gdens, double *gu, double *gamp, void *ws,
                             size_t ws_bytes, void *stream) {
  kbe_status s = check_prop(P, W, G, ws_bytes, ws);
  if (s != KBE_OK) return s;
  if (!gdens || !gu || !gamp) return fail(KBE_EINVAL, "gdens, gu or gamp is NULL");
  return hip_status(kbe::launch_propagate_vjp(P, W, G, gdens, gu, gamp, ws, (hipStream_t)stream),
                    "kbe_propagate_vjp");
}

size_t kbe_propagate_adaptive_workspace(int32_t N, int32_t capacity, int32_t ntau) {
  if (N < 1 || N > KBE_NMAX || capacity < 2 || ntau < 0 || ntau == 1) return 0;
  return kbe::prop_adaptive_ws_bytes(N, capacity, ntau);
}

kbe_status kbe_propagate_adaptive(const kbe_prop *P, const kbe_adapt_ctl *C, const kbe_wts *W,
                                  const kbe_green *G, double *dens, kbe_adapt_trace *trace,
                                  void *ws, size_t ws_bytes, void *stream) {
  kbe_status s = check_green(G, "G");
  if (s != KBE_OK) return s;
  if (!P || !C || !W || !dens || !trace) return fail(KBE_EINVAL, "P, C, W, dens or trace is NULL");
  if (!P->h0 || !P->u) return fail(KBE_EINVAL, "P->h0 or P->u is NULL");
  if (!(P->pulse_sigma > 0)) return fail(KBE_EINVAL, "pulse_sigma = %g <= 0", P->pulse_sigma);
  if (G->nt < 2) return fail(KBE_EINVAL, "capacity nt = %d < 2", G->nt);
  if (!(C->t_end > 0) || !(C->rtol > 0) || !(C->atol > 0) || !(C->h0 > 0))
    return fail(KBE_EINVAL, "t_end, rtol, atol and h0 must be > 0");
  if (C->qmax < 1 || C->qmax > 12) return fail(KBE_EINVAL, "qmax = %d outside 1..12", C->qmax);
  if (C->kmax < 2 || C->kmax > KBE_KMAX)
    return fail(KBE_EINVAL, "kmax = %d outside 2..%d", C->kmax, KBE_KMAX);
  if (C->maxcor < 1 || C->maxcor > 12) return fail(KBE_EINVAL, "maxcor = %d outside 1..12", C->maxcor);
  if (G->ntau > 0 && (!W->wtau || !W->wtau_fwd))
    return fail(KBE_EINVAL, "tau weights are NULL with ntau > 0");
  if (!trace->t || !trace->q || !trace->m || !trace->ks || !trace->err)
    return fail(KBE_EINVAL, "a trace array is NULL");
  const size_t need = kbe_propagate_adaptive_workspace(G->N, G->nt, G->ntau);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  int stalled = 0;
  s = hip_status(kbe::launch_propagate_adaptive(P, C, W, G, dens, trace, ws, (hipStream_t)stream,
                                                &stalled),
                 "kbe_propagate_adaptive");
  if (s != KBE_OK) return s;
  if (stalled == 1)
    return fail(KBE_ESTEP, "step size underflow at t = %.17g after %d points",
                trace->t[trace->nt - 1], trace->nt);
  if (stalled == 2)
    return fail(KBE_ESTEP, "capacity of %d points exhausted at t = %.17g < t_end = %g", G->nt,
                trace->t[trace->nt - 1], C->t_end);
  return s;
}

// ---------------------------------------------------------------------------------------
// Interacting equilibrium initial state.
// ---------------------------------------------------------------------------------------
size_t kbe_equilibrium_workspace(int32_t N, int32_t ntau) {
  if (N < 1 || N > KBE_NMAX || ntau < 2) return 0;
  return kbe::equilibrium_ws_bytes(N, ntau);
}

kbe_status kbe_equilibrium(int32_t N, int32_t ntau, double beta, const double *wtau_fwd,
                           const double *h0, const double *u, kbe_eq_ctl *C, kbe_c128 *mat,
                           void *ws, size_t ws_bytes, void *stream) {
  if (N < 1 || N > KBE_NMAX) return fail(KBE_EINVAL, "N = %d outside 1..%d", N, KBE_NMAX);
  if (ntau < 2) return fail(KBE_EINVAL, "ntau = %d < 2", ntau);
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(KBE_EINVAL, "beta = %g must be > 0", beta);
  if (!wtau_fwd || !h0 || !u || !C || !mat)
    return fail(KBE_EINVAL, "wtau_fwd, h0, u, C or mat is NULL");
  if (!std::isfinite(C->mu)) return fail(KBE_EINVAL, "mu = %g is not finite", C->mu);
  if (!(C->mix > 0.0 && C->mix <= 1.0)) return fail(KBE_EINVAL, "mix = %g outside (0, 1]", C->mix);
  if (!(C->tol > 0.0)) return fail(KBE_EINVAL, "tol = %g must be > 0", C->tol);
  if (C->maxit < 1) return fail(KBE_EINVAL, "maxit = %d < 1", C->maxit);
  const size_t need = kbe::equilibrium_ws_bytes(N, ntau);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  int it = 0;
  double d = 0.0;
  kbe_status s = hip_status(kbe::launch_equilibrium(N, ntau, beta, wtau_fwd, h0, u, C->mu, C->mix,
                                                    C->tol, C->maxit, mat, ws,
                                                    (hipStream_t)stream, &it, &d),
                            "kbe_equilibrium");
  C->iterations = it;
  C->change = d;
  if (s != KBE_OK) return s;
  if (!(d < C->tol))
    return fail(KBE_ECONV, "largest change %.3e >= tol = %.3e after %d iterations", d, C->tol, it);
  return s;
}

// ---------------------------------------------------------------------------------------
// Batches of history rows.
// ---------------------------------------------------------------------------------------
static bool batch_chunk_ok(int32_t chunk) {
  return chunk == 0 || chunk == 32 || chunk == 64 || chunk == 128 || chunk == 256;
}

static kbe_status check_batch(const kbe_batch_item *items, const kbe_batch_item *items_dev,
                              int32_t count, int32_t chunk) {
  if (count < 0 || count > KBE_BATCH_MAX)
    return fail(KBE_ERANGE, "count = %d outside [0, %d]", count, KBE_BATCH_MAX);
  if (!batch_chunk_ok(chunk)) return fail(KBE_EINVAL, "chunk = %d not in {0, 32, 64, 128, 256}", chunk);
  if (count == 0) return ok();
  if (!items || !items_dev) return fail(KBE_EINVAL, "items or items_dev is NULL");
  const unsigned known = KBE_OUT_IR | KBE_OUT_IL | KBE_OUT_ITV;
  for (int32_t i = 0; i < count; ++i) {
    const kbe_batch_item &it = items[i];
    if (it.N < 1 || it.N > KBE_NMAX)
      return fail(KBE_EINVAL, "item %d: N = %d outside 1..%d", i, it.N, KBE_NMAX);
    if (it.flags & ~known) return fail(KBE_EINVAL, "item %d: unknown flag bits 0x%x", i, it.flags);
    if (it.n < 0 || it.m < 0 || it.m > it.n)
      return fail(KBE_ERANGE, "item %d: (n, m) = (%d, %d) needs 0 <= m <= n", i, it.n, it.m);
    if (it.ntau < 0 || it.ntau == 1)
      return fail(KBE_EINVAL, "item %d: ntau = %d (must be 0 or >= 2)", i, it.ntau);
    if (!batch_chunk_ok(it.chunk))
      return fail(KBE_EINVAL, "item %d: chunk = %d not in {0, 32, 64, 128, 256}", i, it.chunk);
    if (it.col_ld < 0)
      return fail(KBE_EINVAL, "item %d: col_ld = %lld < 0", i, (long long)it.col_ld);
    if (it.flags & KBE_OUT_IR) {
      if (!it.IR || !it.sig_ret || !it.col || !it.wn || (it.n > it.m && !it.row))
        return fail(KBE_EINVAL, "item %d: I^R needs IR, sig_ret, col, wn (and row when n > m)", i);
    }
    if (it.flags & KBE_OUT_IL) {
      if (!it.IL || !it.sig_les || !it.rdiag || !it.wm || (it.m > 0 && !it.row))
        return fail(KBE_EINVAL, "item %d: I^< needs IL, sig_les, rdiag, wm (and row when m > 0)", i);
    }
    if (it.flags & KBE_OUT_ITV) {
      if (!it.Itv) return fail(KBE_EINVAL, "item %d: Itv is NULL", i);
      if (it.ntau > 0 && (!it.sig_tv || !it.tv || !it.wtau))
        return fail(KBE_EINVAL, "item %d: I^] needs sig_tv, tv, wtau with ntau > 0", i);
    }
  }
  return ok();
}

size_t kbe_collision_batch_workspace(const kbe_batch_item *items, int32_t count, int32_t chunk) {
  if (count <= 0 || count > KBE_BATCH_MAX || !items || !batch_chunk_ok(chunk)) return 0;
  for (int32_t i = 0; i < count; ++i)
    if (items[i].N < 1 || items[i].N > KBE_NMAX || items[i].m < 0 || items[i].m > items[i].n ||
        items[i].ntau < 0 || !batch_chunk_ok(items[i].chunk))
      return 0;
  return kbe::batch_ws_bytes(items, count, chunk);
}

kbe_status kbe_collision_batch(const kbe_batch_item *items, const kbe_batch_item *items_dev,
                               int32_t count, int32_t chunk, void *ws, size_t ws_bytes,
                               void *stream) {
  kbe_status s = check_batch(items, items_dev, count, chunk);
  if (s != KBE_OK || count == 0) return s;
  const size_t need = kbe::batch_ws_bytes(items, count, chunk);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  return hip_status(kbe::launch_batch(items, items_dev, count, chunk, ws, (hipStream_t)stream),
                    "kbe_collision_batch");
}

}  // extern "C"

namespace {
// Event pair for the tuners, destroyed with the object.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t init() {
    hipError_t e = hipEventCreate(&a);
    return e == hipSuccess ? hipEventCreate(&b) : e;
  }
  ~EventPair() {
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
  }
};

// One warm-up call, then `reps` timed calls; *ms = the fastest.
hipError_t time_batch(const kbe_batch_item *items, const kbe_batch_item *items_dev, int count,
                      int chunk, void *ws, hipStream_t st, EventPair &ev, int reps, float *ms) {
  hipError_t err = kbe::launch_batch(items, items_dev, count, chunk, ws, st);
  *ms = -1.0f;
  for (int r = 0; r < reps && err == hipSuccess; ++r) {
    err = hipEventRecord(ev.a, st);
    if (err == hipSuccess) err = kbe::launch_batch(items, items_dev, count, chunk, ws, st);
    if (err == hipSuccess) err = hipEventRecord(ev.b, st);
    if (err == hipSuccess) err = hipEventSynchronize(ev.b);
    float t = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, ev.a, ev.b);
    if (err == hipSuccess && (*ms < 0.0f || t < *ms)) *ms = t;
  }
  return err;
}

int floor_log2(int64_t x) {
  int b = 0;
  while (x > 1) {
    x >>= 1;
    ++b;
  }
  return b;
}
}  // namespace

extern "C" {

static kbe_status check_batch_vjp(const kbe_batch_vjp_item *items,
                                  const kbe_batch_vjp_item *items_dev, int32_t count) {
  if (count < 0 || count > KBE_BATCH_MAX)
    return fail(KBE_ERANGE, "count = %d outside [0, %d]", count, KBE_BATCH_MAX);
  if (count == 0) return ok();
  if (!items || !items_dev) return fail(KBE_EINVAL, "items or items_dev is NULL");
  const unsigned known = KBE_OUT_IR | KBE_OUT_IL | KBE_OUT_ITV;
  for (int32_t i = 0; i < count; ++i) {
    const kbe_batch_vjp_item &v = items[i];
    const kbe_batch_item &it = v.row;
    if (it.N < 1 || it.N > KBE_NMAX)
      return fail(KBE_EINVAL, "item %d: N = %d outside 1..%d", i, it.N, KBE_NMAX);
    if (it.flags & ~known) return fail(KBE_EINVAL, "item %d: unknown flag bits 0x%x", i, it.flags);
    if (it.n < 0 || it.m < 0 || it.m > it.n)
      return fail(KBE_ERANGE, "item %d: (n, m) = (%d, %d) needs 0 <= m <= n", i, it.n, it.m);
    if (it.ntau < 0 || it.ntau == 1)
      return fail(KBE_EINVAL, "item %d: ntau = %d (must be 0 or >= 2)", i, it.ntau);
    if (it.col_ld < 0)
      return fail(KBE_EINVAL, "item %d: col_ld = %lld < 0", i, (long long)it.col_ld);
    if (!v.g_sig_ret || !v.g_sig_les || !v.g_col || !v.g_row || !v.g_rdiag ||
        (it.ntau > 0 && (!v.g_sig_tv || !v.g_tv)))
      return fail(KBE_EINVAL, "item %d: a gradient array is NULL", i);
    if (it.flags & KBE_OUT_IR) {
      if (!v.gIR || !it.sig_ret || !it.col || !it.wn || (it.n > it.m && !it.row))
        return fail(KBE_EINVAL, "item %d: I^R needs gIR, sig_ret, col, wn (and row when n > m)", i);
    }
    if (it.flags & KBE_OUT_IL) {
      if (!v.gIL || !it.sig_les || !it.rdiag || !it.wm || (it.m > 0 && !it.row))
        return fail(KBE_EINVAL, "item %d: I^< needs gIL, sig_les, rdiag, wm (and row when m > 0)", i);
    }
    if ((it.flags & KBE_OUT_ITV) && it.ntau > 0) {
      if (!v.gItv || !it.sig_tv || !it.tv || !it.wtau)
        return fail(KBE_EINVAL, "item %d: I^] needs gItv, sig_tv, tv, wtau with ntau > 0", i);
    }
  }
  return ok();
}

size_t kbe_collision_batch_vjp_workspace(int32_t count) {
  if (count < 0 || count > KBE_BATCH_MAX) return 0;
  return kbe::batch_vjp_ws_bytes(count);
}

kbe_status kbe_collision_batch_vjp(const kbe_batch_vjp_item *items,
                                   const kbe_batch_vjp_item *items_dev, int32_t count, void *ws,
                                   size_t ws_bytes, void *stream) {
  kbe_status s = check_batch_vjp(items, items_dev, count);
  if (s != KBE_OK || count == 0) return s;
  const size_t need = kbe::batch_vjp_ws_bytes(count);
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  return hip_status(kbe::launch_batch_vjp(items_dev, count, ws, (hipStream_t)stream),
                    "kbe_collision_batch_vjp");
}

kbe_status kbe_collision_batch_tune(const kbe_batch_item *items, const kbe_batch_item *items_dev,
                                    int32_t count, void *ws, size_t ws_bytes, void *stream,
                                    int32_t *best_chunk, float *times_ms) {
  kbe_status s = check_batch(items, items_dev, count, 0);
  if (s != KBE_OK) return s;
  if (!best_chunk) return fail(KBE_EINVAL, "best_chunk is NULL");
  static const int cand[4] = {32, 64, 128, 256};
  *best_chunk = kbe::batch_default_chunk();
  if (count == 0) return ok();
  const size_t need = kbe::batch_ws_bytes(items, count, 32);  // the largest requirement
  if (!ws || ws_bytes < need) return fail(KBE_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  EventPair ev;
  hipError_t err = ev.init();
  float best = -1.0f;
  for (int k = 0; k < 4 && err == hipSuccess; ++k) {
    float ms = 0.0f;
    err = time_batch(items, items_dev, count, cand[k], ws, st, ev, 1, &ms);
    if (err != hipSuccess) break;
    if (times_ms) times_ms[k] = ms;
    if (best < 0.0f || ms < best) {
      best = ms;
      *best_chunk = cand[k];
    }
  }
  return hip_status(err, "kbe_collision_batch_tune");
}

kbe_status kbe_collision_batch_tune_groups(kbe_batch_item *items, kbe_batch_item *items_dev,
                                           int32_t count, void *ws, size_t ws_bytes, void *stream,
                                           float *best_ms) {
  int32_t c0 = 0;
  kbe_status s = kbe_collision_batch_tune(items, items_dev, count, ws, ws_bytes, stream, &c0, nullptr);
  if (s != KBE_OK) return s;
  if (best_ms) *best_ms = 0.0f;
  if (count == 0) return ok();
  hipStream_t st = (hipStream_t)stream;
  const size_t isz = sizeof(kbe_batch_item) * (size_t)count;
  auto upload = [&]() {
    hipError_t e = hipMemcpyAsync(items_dev, items, isz, hipMemcpyHostToDevice, st);
    return e == hipSuccess ? hipStreamSynchronize(st) : e;
  };
  EventPair ev;
  hipError_t err = ev.init();
  for (int32_t i = 0; i < count; ++i) items[i].chunk = c0;
  if (err == hipSuccess) err = upload();
  float cur = 0.0f;
  if (err == hipSuccess) err = time_batch(items, items_dev, count, 0, ws, st, ev, 3, &cur);
  static const int cand[4] = {32, 64, 128, 256};
  // One coordinate-descent pass over the groups of a key, heaviest group first (by the blocks
  // its items read): each other chunk is tried on the group alone and kept if the whole call
  // gets more than 1% faster.
  std::vector<int64_t> key(count);
  auto pass = [&](bool by_length) {
    std::vector<std::pair<double, int64_t>> weight;
    for (int32_t i = 0; i < count; ++i) {
      const kbe_batch_item &it = items[i];
      key[i] = (int64_t)it.N * 64 + (by_length ? floor_log2((int64_t)it.n + 1) : 0);
      const double w = (double)it.N * it.N * (2.0 * it.n + it.m + it.ntau + 4);
      bool found = false;
      for (auto &g : weight)
        if (g.second == key[i]) {
          g.first += w;
          found = true;
        }
      if (!found) weight.push_back({w, key[i]});
    }
    std::sort(weight.begin(), weight.end(),
              [](const std::pair<double, int64_t> &a, const std::pair<double, int64_t> &b) {
                return a.first > b.first;
              });
    auto set_group = [&](int64_t g, int32_t c) {
      for (int32_t i = 0; i < count; ++i)
        if (key[i] == g) items[i].chunk = c;
    };
    for (const auto &g : weight) {
      if (err != hipSuccess) break;
      int32_t keep = c0;
      for (int32_t i = 0; i < count; ++i)
        if (key[i] == g.second) {
          keep = items[i].chunk;  // the group's chunk so far (one value per group)
          break;
        }
      const int32_t start = keep;
      for (int k = 0; k < 4 && err == hipSuccess; ++k) {
        if (cand[k] == start) continue;
        set_group(g.second, cand[k]);
        err = upload();
        float t = 0.0f;
        if (err == hipSuccess) err = time_batch(items, items_dev, count, 0, ws, st, ev, 3, &t);
        if (err == hipSuccess && t < 0.99f * cur) {
          cur = t;
          keep = cand[k];
        }
      }
      set_group(g.second, keep);
    }
  };
  pass(false);  // by N
  pass(true);   // by N and length bucket
  if (err == hipSuccess) err = upload();
  if (best_ms) *best_ms = cur;
  return hip_status(err, "kbe_collision_batch_tune_groups");
}

}  // extern "C"
