// History integrals of arXiv:2405.08737 (Eq. KBE2 lesser form, history terms of Eq. KBE3) and
// their adjoint, on gfx950.
//
// Every output block is a sum over terms t of a block product with a scalar weight,
//   OP_N : c Q_t P_t,   OP_H : c Q_t P_t^dagger,   OP_HN : c Q_t^dagger P_t,
// where P_t is a block of the large Green's-function storage streamed from HBM and Q_t a block
// of a small, cache-resident operand (self-energy row or cotangent).  A family of such terms
// ("class") is indexed so that Q depends on the term index t only: outputs that share a term
// index share Q.  The weight and P depend on (output, t); some Matsubara terms carry two
// (c, P) pairs, which are combined before the product.
//
// Work decomposition: the term index is cut into chunks of SC terms; a wavefront computes the
// partial sums of MO consecutive outputs over one chunk (MO = 4 on the MFMA path, so each Q
// load serves four P blocks) and writes them to the workspace; a reduce kernel adds the chunks
// of every output in a fixed order, so results are deterministic (no floating-point atomics).
// Workgroups are laid out chunk-fastest and every class starts on a multiple of 8 workgroups:
// with round-robin dispatch over the 8 XCDs, all tasks of a chunk land on one XCD and its L2
// holds that chunk's Q blocks.
//
// Implementations of a task:
//   * task_mfma16 (N = 16): FP64 matrix cores.  A 16x16 complex block product is four real
//     products of four v_mfma_f64_16x16x4 k-slices each; two accumulators per output (real and
//     imaginary part) with the negated imaginary part of Q prepared once per term.  Operands go
//     from global memory straight into the MFMA register layouts: the B operand (lane l holds
//     B[k][l%16], k = 4*slice + l/16) is a contiguous 1 KiB row-slice of a row-major block, the
//     A operand (lane l holds A[l%16][k]) reads 64-byte row segments.
//   * task_generic (any N <= 16): vector ALU, one output per wave, one output element per lane,
//     several terms per wave for small N summed across lanes at the end.
#include "kbe_dev.h"
#include "kbe_internal.h"

#include <initializer_list>

namespace kbe {

enum Cls {
  C_IRC,   // I^R, s <= m:  w[n][s] Sigma^R(s) kp[s][m]               (G^<(s,m) stored)
  C_IRR,   // I^R, s > m : -w[n][s] Sigma^R(s) kp[m][s]^dagger        (G^<(s,m) = -kp[m][s]^dag)
  C_IL,    // I^<, s <= m:  w[m][s] Sigma^<(s) G^R(m,s)^dagger
  C_ITV,   // I^]:  -i wtau[j] Sigma^](j) tv[m][J-j]^dagger
  C_JR,    // J^] real-time part:  w[n][s] Sigma^R(s) tv[s][j]
  C_JM,    // J^] Matsubara part, split at tau_j
  B_R1,    // adjoint: gSigma^R(s) from C_IRC terms
  B_R2,    // adjoint: gSigma^R(s) from C_IRR terms
  B_R3,    // adjoint: gSigma^R(s) from C_JR terms
  B_L,     // adjoint: gSigma^<(s) from C_IL terms
  B_T1,    // adjoint: gSigma^](j) from C_ITV terms
  B_T2,    // adjoint: gSigma^](l) from C_JM terms
  G_MAT,   // adjoint: gG^M(k) from C_JM terms
  NCLS
};
enum Op { OP_N = 0, OP_H = 1, OP_HN = 2 };

template <int CLS>
__host__ __device__ constexpr int cls_op() {
  return (CLS == C_IRR || CLS == C_IL || CLS == C_ITV || CLS == B_R1 || CLS == B_R3 || CLS == B_T2)
             ? OP_H
             : (CLS == G_MAT ? OP_HN : OP_N);
}

// Term-index range [lo, hi) of output o.
template <int CLS>
__device__ __forceinline__ void cls_range(const Params &p, int o, int &lo, int &hi) {
  const int m = p.m0 + o;
  switch (CLS) {
    case C_IRC: lo = 0; hi = m + 1; break;
    case C_IRR: lo = m + 1; hi = p.n + 1; break;
    case C_IL: lo = 0; hi = m + 1; break;
    case C_ITV: lo = 0; hi = p.ntau; break;
    case C_JR: lo = 0; hi = p.n + 1; break;
    case C_JM: lo = 0; hi = p.ntau; break;
    case B_R1: lo = o > p.m0 ? o : p.m0; hi = p.m1; break;
    case B_R2: lo = p.m0; hi = o < p.m1 ? o : p.m1; break;
    case B_R3: lo = 0; hi = p.ntau; break;
    case B_L: lo = o > p.m0 ? o : p.m0; hi = p.m1; break;
    case B_T1: lo = p.m0; hi = p.m1; break;
    case B_T2: lo = 0; hi = p.ntau; break;
    case G_MAT: lo = 0; hi = p.ntau; break;
  }
}

// Shared operand of term t.
template <int CLS>
__device__ __forceinline__ const kbe_c128 *cls_Q(const Params &p, int t) {
  const int64_t E = bsz(p);
  switch (CLS) {
    case C_IRC: case C_IRR: case C_JR: return p.ret + t * E;
    case C_IL: return p.les + t * E;
    case C_ITV: case C_JM: case G_MAT: return p.stv + t * E;
    case B_R1: case B_R2: return p.gIR + (t - p.m0) * E;
    case B_L: return p.gIL + (t - p.m0) * E;
    case B_T1: return p.gItv + (t - p.m0) * E;
    case B_R3: case B_T2: return p.gJ + t * E;
  }
  return nullptr;
}

// Weight(s) and streamed block(s) of term t of output o (t inside o's range): returns 1 or 2
// pairs (c0, P0), (c1, P1).  Two-piece terms are assembled with selects, which keeps the pairs
// in registers.
__device__ __forceinline__ int two_pieces(bool va, cd ca, const kbe_c128 *pa, bool vb, cd cb,
                                          const kbe_c128 *pb, cd &c0, const kbe_c128 *&P0,
                                          cd &c1, const kbe_c128 *&P1) {
  c0 = va ? ca : cb;
  P0 = va ? pa : pb;
  c1 = cb;
  P1 = pb;
  return (va ? 1 : 0) + (vb ? 1 : 0);
}

template <int CLS>
__device__ __forceinline__ int cls_P(const Params &p, int o, int t, cd &c0, const kbe_c128 *&P0,
                                     cd &c1, const kbe_c128 *&P1) {
  const int64_t E = bsz(p);
  const int J = p.J, m = p.m0 + o;
  switch (CLS) {
    case C_IRC: c0 = {p.w[(int64_t)p.n * p.nt + t], 0.0}; P0 = kp_blk(p, t, m); return 1;
    case C_IRR: c0 = {-p.w[(int64_t)p.n * p.nt + t], 0.0}; P0 = kp_blk(p, m, t); return 1;
    case C_IL:
      c0 = {p.w[(int64_t)m * p.nt + t], 0.0};
      P0 = t < m ? kp_blk(p, m, t) : p.rdiag + m * E;
      return 1;
    case C_ITV: c0 = {0.0, -p.wtau[t]}; P0 = tv_blk(p, m, J - t); return 1;
    case C_JR: c0 = {p.w[(int64_t)p.n * p.nt + t], 0.0}; P0 = tv_blk(p, t, o); return 1;
    case C_JM:    // l = t, j = o: [0,tau_j] uses -G^M(beta+tau_l-tau_j), [tau_j,beta] G^M(tau_l-tau_j)
    case B_T2: {  // j = t, l = o: the same pairs seen from the self-energy side
      const int l = CLS == C_JM ? t : o, j = CLS == C_JM ? o : t;
      const bool va = l <= j, vb = l >= j;
      const cd ca = {va ? -p.wf[(int64_t)j * p.ntau + l] : 0.0, 0.0};
      const cd cb = {vb ? p.wf[(int64_t)(J - j) * p.ntau + (J - l)] : 0.0, 0.0};
      return two_pieces(va, ca, p.mat + (va ? J + l - j : 0) * E, vb, cb,
                        p.mat + (vb ? l - j : 0) * E, c0, P0, c1, P1);
    }
    case B_R1: c0 = {p.w[(int64_t)p.n * p.nt + o], 0.0}; P0 = kp_blk(p, o, t); return 1;
    case B_R2: c0 = {-p.w[(int64_t)p.n * p.nt + o], 0.0}; P0 = kp_blk(p, t, o); return 1;
    case B_R3: c0 = {p.w[(int64_t)p.n * p.nt + o], 0.0}; P0 = tv_blk(p, o, t); return 1;
    case B_L:
      c0 = {p.w[(int64_t)t * p.nt + o], 0.0};
      P0 = t > o ? kp_blk(p, t, o) : p.rdiag + o * E;
      return 1;
    case B_T1: c0 = {0.0, p.wtau[o]}; P0 = tv_blk(p, t, J - o); return 1;
    case G_MAT: {  // l = t, k = o: pairs with j - l = J - k (l <= k) or l - j = k (l >= k)
      const int l = t, kk = o;
      const bool va = l <= kk, vb = l >= kk;
      const int ja = va ? l + J - kk : 0, jb = vb ? l - kk : 0;
      const cd ca = {va ? -p.wf[(int64_t)ja * p.ntau + l] : 0.0, 0.0};
      const cd cb = {vb ? p.wf[(int64_t)(J - jb) * p.ntau + (J - l)] : 0.0, 0.0};
      return two_pieces(va, ca, p.gJ + ja * E, vb, cb, p.gJ + jb * E, c0, P0, c1, P1);
    }
  }
  return 0;
}

__device__ __forceinline__ void range_rt(int cls, const Params &p, int o, int &lo, int &hi) {
  switch (cls) {
    case C_IRC: cls_range<C_IRC>(p, o, lo, hi); break;
    case C_IRR: cls_range<C_IRR>(p, o, lo, hi); break;
    case C_IL: cls_range<C_IL>(p, o, lo, hi); break;
    case C_ITV: cls_range<C_ITV>(p, o, lo, hi); break;
    case C_JR: cls_range<C_JR>(p, o, lo, hi); break;
    case C_JM: cls_range<C_JM>(p, o, lo, hi); break;
    case B_R1: cls_range<B_R1>(p, o, lo, hi); break;
    case B_R2: cls_range<B_R2>(p, o, lo, hi); break;
    case B_R3: cls_range<B_R3>(p, o, lo, hi); break;
    case B_L: cls_range<B_L>(p, o, lo, hi); break;
    case B_T1: cls_range<B_T1>(p, o, lo, hi); break;
    case B_T2: cls_range<B_T2>(p, o, lo, hi); break;
    case G_MAT: cls_range<G_MAT>(p, o, lo, hi); break;
    default: lo = hi = 0;
  }
}

// ------------------------------------------------------------------------------------------
// Generic vector-ALU task: one output o, terms t in [t0, t1).  For N*N <= 64 the wave runs
// G = 64/(N*N) groups of N*N lanes over interleaved terms (lane = one output element) and sums
// the groups with cross-lane shuffles; for larger N each lane owns up to 4 elements.
// ------------------------------------------------------------------------------------------
template <int CLS>
__device__ __forceinline__ void task_generic(const Params &p, int o, int t0, int t1,
                                             kbe_c128 *out, int lane) {
  constexpr int OP = cls_op<CLS>();
  const int N = p.N, E = N * N;
  const int Gs = E <= 64 ? 64 / E : 1;
  const int g = E <= 64 ? lane / E : 0;
  const int R = E <= 64 ? 1 : (E + 63) / 64;
  cd acc[4] = {czero(), czero(), czero(), czero()};
  if (g < Gs) {
    for (int t = t0 + g; t < t1; t += Gs) {
      const kbe_c128 *Q = cls_Q<CLS>(p, t);
      cd c0, c1;
      const kbe_c128 *P0, *P1;
      const int np = cls_P<CLS>(p, o, t, c0, P0, c1, P1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r >= R) break;
        const int e = E <= 64 ? lane % E : lane + 64 * r;
        if (e >= E) break;
        const int i = e / N, j = e % N;
        for (int u = 0; u < np; ++u) {
          const kbe_c128 *Pu = u == 0 ? P0 : P1;
          cd s = czero();
          for (int k = 0; k < N; ++k) {
            if (OP == OP_N) s = s + ld(Q + i * N + k) * ld(Pu + k * N + j);
            else if (OP == OP_H) s = s + ld(Q + i * N + k) * cj(ld(Pu + j * N + k));
            else s = s + cj(ld(Q + k * N + i)) * ld(Pu + k * N + j);
          }
          acc[r] = acc[r] + (u == 0 ? c0 : c1) * s;
        }
      }
    }
  }
  if (E <= 64) {
    cd tot = acc[0];
    for (int q = 1; q < Gs; ++q) {  // uniform across the wave
      const int src = lane + q * E < 64 ? lane + q * E : lane;
      const double re = __shfl(acc[0].re, src), im = __shfl(acc[0].im, src);
      if (lane < E) tot = tot + cd{re, im};
    }
    if (lane < E) st(out + lane, tot);
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = lane + 64 * r;
      if (r < R && e < E) st(out + e, acc[r]);
    }
  }
}

// ------------------------------------------------------------------------------------------
// FP64 MFMA task (N = 16): outputs o0..o0+no-1 (no <= MO), terms t in [t0, t1).
// The weight goes on the streamed block: P' = c P (OP_N, OP_HN) or conj(c) P (OP_H), so that
//   OP_N : out = sum Q P'        A = Q  (row segments),  B = P' (row slices)
//   OP_H : out = (sum P' Q^dag)^dag   A = P' (row segments), B = Q^dag (Q row segments)
//   OP_HN: out = sum Q^dag P'    A = Q^dag (Q row slices),   B = P' (row slices)
// With (ar, ai) / (br, bi) the parts of the A / B operands and x' = -x for the part that
// enters with a minus sign, each output keeps  re += ar br - ai bi,  im += ar bi + ai br.
// D layout of v_mfma_f64_16x16x4 (checked on gfx950): lane l, register r holds element
// (l/16 + 4*r, l%16).
// ------------------------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int CLS, int MO>
__device__ __forceinline__ void task_mfma16(const Params &p, int o0, int no, int t0, int t1,
                                            kbe_c128 *const *out, int lane) {
  constexpr int OP = cls_op<CLS>();
  const int row = lane & 15, q = lane >> 4;
  const int offA = row * 16 + q;  // element (row, 4*slice + q): + 4*slice
  const int offB = q * 16 + row;  // element (4*slice + q, row): + 64*slice
  v4d are[MO], aim[MO];
  int lo[MO], hi[MO];
#pragma unroll
  for (int u = 0; u < MO; ++u) {
    are[u] = v4d{0, 0, 0, 0};
    aim[u] = are[u];
    lo[u] = 0;
    hi[u] = 0;
    if (u < no) cls_range<CLS>(p, o0 + u, lo[u], hi[u]);
  }
  for (int t = t0; t < t1; ++t) {
    const kbe_c128 *Q = cls_Q<CLS>(p, t);
    double qr[4], qi[4], nqi[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      const cd v = ld(Q + (OP == OP_HN ? offB + 64 * sl : offA + 4 * sl));
      qr[sl] = v.re;
      qi[sl] = v.im;
      nqi[sl] = -v.im;
    }
#pragma unroll
    for (int u = 0; u < MO; ++u) {
      if (u >= no || t < lo[u] || t >= hi[u]) continue;  // wave-uniform
      cd c0, c1;
      const kbe_c128 *P0, *P1;
      const int np = cls_P<CLS>(p, o0 + u, t, c0, P0, c1, P1);
      if (OP == OP_H) {
        c0 = cj(c0);
        c1 = cj(c1);
      }
      cd pv[4];
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        const int off = OP == OP_H ? offA + 4 * sl : offB + 64 * sl;
        pv[sl] = c0 * ld(P0 + off);
        if (np > 1) pv[sl] = pv[sl] + c1 * ld(P1 + off);
      }
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        if (OP == OP_N) {  // A = Q, B = P'
          are[u] = mfma(qr[sl], pv[sl].re, are[u]);
          are[u] = mfma(nqi[sl], pv[sl].im, are[u]);
          aim[u] = mfma(qr[sl], pv[sl].im, aim[u]);
          aim[u] = mfma(qi[sl], pv[sl].re, aim[u]);
        } else if (OP == OP_H) {  // A = P', B = Q^dag: br = qr, bi = -qi
          are[u] = mfma(pv[sl].re, qr[sl], are[u]);
          are[u] = mfma(pv[sl].im, qi[sl], are[u]);
          aim[u] = mfma(pv[sl].re, nqi[sl], aim[u]);
          aim[u] = mfma(pv[sl].im, qr[sl], aim[u]);
        } else {  // A = Q^dag: ar = qr, ai = -qi; B = P'
          are[u] = mfma(qr[sl], pv[sl].re, are[u]);
          are[u] = mfma(qi[sl], pv[sl].im, are[u]);
          aim[u] = mfma(qr[sl], pv[sl].im, aim[u]);
          aim[u] = mfma(nqi[sl], pv[sl].re, aim[u]);
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < MO; ++u) {
    if (u >= no || hi[u] <= t0 || lo[u] >= t1) continue;  // no term of this chunk: not written
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = q + 4 * r;
      if (OP == OP_H) st(out[u] + row * 16 + i, cd{are[u][r], -aim[u][r]});
      else st(out[u] + i * 16 + row, cd{are[u][r], aim[u][r]});
    }
  }
}

// One launch covers every class of a call.  Class k owns workgroups [first_wg[k],
// first_wg[k+1]) (a multiple of 8 apart); local workgroup lb handles chunk lb % nchunk and
// output groups 4*(lb / nchunk) + wave, each of MO outputs.
struct FusedPlan {
  int ncls, SC, MO;
  int cls[8], nout[8], nchunk[8], ngroup[8];
  int64_t first_wg[9];
  int64_t off[8];  // byte offset of each class's partials [nchunk][nout][N*N] in the workspace
};

template <bool MFMA, int CLS>
__device__ __forceinline__ void run_task(const Params &p, const FusedPlan &pl, int k, int64_t lb,
                                         char *ws, int lane, int wave) {
  const int nch = pl.nchunk[k];
  const int ch = (int)(lb % nch);
  const int g = (int)(lb / nch) * 4 + wave;
  if (g >= pl.ngroup[k]) return;
  const int t0 = ch * pl.SC, t1 = t0 + pl.SC;
  kbe_c128 *base = (kbe_c128 *)(ws + pl.off[k]);
  const int64_t E = bsz(p);
  if (MFMA) {
    constexpr int MO = 4;
    const int o0 = g * MO;
    const int no = pl.nout[k] - o0 < MO ? pl.nout[k] - o0 : MO;
    int lo = 1 << 30, hi = 0;  // union of the outputs' ranges, clipped to the chunk
    kbe_c128 *out[MO];
#pragma unroll
    for (int u = 0; u < MO; ++u) {
      out[u] = base + ((int64_t)ch * pl.nout[k] + o0 + (u < no ? u : 0)) * E;
      if (u < no) {
        int a, b;
        cls_range<CLS>(p, o0 + u, a, b);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
      }
    }
    const int a = t0 > lo ? t0 : lo, b = t1 < hi ? t1 : hi;
    if (a >= b) return;
    task_mfma16<CLS, MO>(p, o0, no, a, b, out, lane);
  } else {
    const int o = g;
    int lo, hi;
    cls_range<CLS>(p, o, lo, hi);
    const int a = t0 > lo ? t0 : lo, b = t1 < hi ? t1 : hi;
    if (a >= b) return;
    task_generic<CLS>(p, o, a, b, base + ((int64_t)ch * pl.nout[k] + o) * E, lane);
  }
}

template <bool MFMA>
__global__ void __launch_bounds__(256) stream_fused(Params p, FusedPlan pl, char *ws) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t b = blockIdx.x;
  if (b >= pl.first_wg[pl.ncls]) return;  // no block-level barriers anywhere below
  int k = 0;
  while (b >= pl.first_wg[k + 1]) ++k;
  const int64_t lb = b - pl.first_wg[k];
  switch (pl.cls[k]) {
    case C_IRC: run_task<MFMA, C_IRC>(p, pl, k, lb, ws, lane, wave); break;
    case C_IRR: run_task<MFMA, C_IRR>(p, pl, k, lb, ws, lane, wave); break;
    case C_IL: run_task<MFMA, C_IL>(p, pl, k, lb, ws, lane, wave); break;
    case C_ITV: run_task<MFMA, C_ITV>(p, pl, k, lb, ws, lane, wave); break;
    case C_JR: run_task<MFMA, C_JR>(p, pl, k, lb, ws, lane, wave); break;
    case C_JM: run_task<MFMA, C_JM>(p, pl, k, lb, ws, lane, wave); break;
    case B_R1: run_task<MFMA, B_R1>(p, pl, k, lb, ws, lane, wave); break;
    case B_R2: run_task<MFMA, B_R2>(p, pl, k, lb, ws, lane, wave); break;
    case B_R3: run_task<MFMA, B_R3>(p, pl, k, lb, ws, lane, wave); break;
    case B_L: run_task<MFMA, B_L>(p, pl, k, lb, ws, lane, wave); break;
    case B_T1: run_task<MFMA, B_T1>(p, pl, k, lb, ws, lane, wave); break;
    case B_T2: run_task<MFMA, B_T2>(p, pl, k, lb, ws, lane, wave); break;
    case G_MAT: run_task<MFMA, G_MAT>(p, pl, k, lb, ws, lane, wave); break;
  }
}

// out[x] (=|+=) the sum, in increasing chunk order, of the chunks of up to three classes'
// partial arrays that intersect output o's term range.
struct RedIn {
  const kbe_c128 *a[3];
  int cls[3], nchunk[3];
  int nparts, SC;
};
__global__ void __launch_bounds__(256) reduce_kernel(Params p, RedIn in, int nout,
                                                     kbe_c128 *out, int accumulate) {
  const int64_t E = bsz(p);
  const int64_t nel = (int64_t)nout * E;
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nel) return;
  const int o = (int)(x / E);
  cd s = czero();
  for (int k = 0; k < in.nparts; ++k) {
    int lo, hi;
    range_rt(in.cls[k], p, o, lo, hi);
    if (hi <= lo) continue;
    const int c0 = lo / in.SC;
    int c1 = (hi - 1) / in.SC;
    if (c1 > in.nchunk[k] - 1) c1 = in.nchunk[k] - 1;
    for (int c = c0; c <= c1; ++c) s = s + ld(in.a[k] + (int64_t)c * nel + x);
  }
  if (accumulate) s = s + ld(out + x);
  st(out + x, s);
}

// ------------------------------------------------------------------------------------------
// Adjoint, Green's-function part: every gradient block is a sum of at most two products
// c X^dagger Y of small operands (the forward's self-energy row and the cotangents):
//   kp[a][b], a <= b:  w[n][a] Sigma^R(a)^dag gIR(b)            (b in range; from C_IRC)
//                    - w[n][b] gIR(a)^dag Sigma^R(b)            (a in range, a < b; C_IRR)
//   kp[a][b], a > b :  w[a][b] gIL(a)^dag Sigma^<(b)            (a in range; C_IL)
//   rdiag[a]        :  w[a][a] gIL(a)^dag Sigma^<(a)            (a in range; C_IL)
//   tv[s][k]        :  w[n][s] Sigma^R(s)^dag gJ(k)              (C_JR)
//                    - i wtau[J-k] gItv(s)^dag Sigma^](J-k)     (s in range; C_ITV)
// Blocks with no term are not written.
// ------------------------------------------------------------------------------------------
struct GT {
  cd c;
  const kbe_c128 *X, *Y;
};

// kind 0: kp block (a, b); kind 1: rdiag[a]; kind 2: tv[a][b].  Returns the number of terms
// (0..2) in t0, t1 (two named terms rather than an array, to keep them in registers).
__device__ __forceinline__ int grad_terms(const Params &p, int kind, int a, int b, GT &t0, GT &t1,
                                          kbe_c128 *&dst) {
  const int64_t E = bsz(p);
  int nt = 0;
  const bool ina = a >= p.m0 && a < p.m1, inb = b >= p.m0 && b < p.m1;
  auto push = [&](GT v) {
    if (nt == 0) t0 = v;
    else t1 = v;
    ++nt;
  };
  if (kind == 0) {
    dst = p.gkp + ((int64_t)a * p.ldt + b) * E;
    if (a <= b) {
      if (p.fIR && inb) push({{p.w[(int64_t)p.n * p.nt + a], 0.0}, p.ret + a * E, p.gIR + (b - p.m0) * E});
      if (p.fIR && ina && a < b)
        push({{-p.w[(int64_t)p.n * p.nt + b], 0.0}, p.gIR + (a - p.m0) * E, p.ret + b * E});
    } else if (p.fIL && ina) {
      push({{p.w[(int64_t)a * p.nt + b], 0.0}, p.gIL + (a - p.m0) * E, p.les + b * E});
    }
  } else if (kind == 1) {
    dst = p.grdiag + a * E;
    if (p.fIL && ina) push({{p.w[(int64_t)a * p.nt + a], 0.0}, p.gIL + (a - p.m0) * E, p.les + a * E});
  } else {
    dst = p.gtv + ((int64_t)a * p.ntau + b) * E;
    if (p.fJTV) push({{p.w[(int64_t)p.n * p.nt + a], 0.0}, p.ret + a * E, p.gJ + b * E});
    if (p.fITV && ina)
      push({{0.0, -p.wtau[p.J - b]}, p.gItv + (a - p.m0) * E, p.stv + (p.J - b) * E});
  }
  return nt;
}

__device__ __forceinline__ void grad_block_index(const Params &p, int64_t blk, int &kind, int &a,
                                                 int &b) {
  const int64_t n1 = p.n + 1;
  if (blk < n1 * n1) {
    kind = 0;
    a = (int)(blk / n1);
    b = (int)(blk % n1);
  } else if (blk < n1 * n1 + n1) {
    kind = 1;
    a = (int)(blk - n1 * n1);
    b = a;
  } else {
    const int64_t k = blk - n1 * n1 - n1;
    kind = 2;
    a = (int)(k / p.ntau);
    b = (int)(k % p.ntau);
  }
}

__global__ void __launch_bounds__(256) grad_generic(Params p, int64_t nblk) {
  const int E = p.N * p.N;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t blk = gid / E;
  if (blk >= nblk) return;
  const int e = (int)(gid % E), i = e / p.N, j = e % p.N;
  int kind, a, b;
  grad_block_index(p, blk, kind, a, b);
  GT t0, t1;
  kbe_c128 *dst;
  const int nt = grad_terms(p, kind, a, b, t0, t1, dst);
  if (nt == 0) return;
  cd s = czero();
  for (int q = 0; q < nt; ++q) {
    const GT &tq = q == 0 ? t0 : t1;
    cd x = czero();
    for (int k = 0; k < p.N; ++k) x = x + cj(ld(tq.X + k * p.N + i)) * ld(tq.Y + k * p.N + j);
    s = s + tq.c * x;
  }
  if (!p.overwrite) s = s + ld(dst + e);
  st(dst + e, s);
}

__global__ void __launch_bounds__(256) grad_mfma16(Params p, int64_t nblk) {
  const int lane = threadIdx.x & 63;
  const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blk >= nblk) return;
  int kind, a, b;
  grad_block_index(p, blk, kind, a, b);
  GT t0, t1;
  kbe_c128 *dst;
  const int nt = grad_terms(p, kind, a, b, t0, t1, dst);
  if (nt == 0) return;
  const int row = lane & 15, q = lane >> 4;
  const int offB = q * 16 + row;
  v4d rr = {0, 0, 0, 0}, ii = rr, ri = rr, ir = rr;
  for (int u = 0; u < nt; ++u) {
    const GT &tu = u == 0 ? t0 : t1;
    cd xa[4], yb[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      xa[sl] = cj(tu.c) * ld(tu.X + offB + 64 * sl);
      yb[sl] = ld(tu.Y + offB + 64 * sl);
    }
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      rr = mfma(xa[sl].re, yb[sl].re, rr);
      ii = mfma(xa[sl].im, yb[sl].im, ii);
      ri = mfma(xa[sl].re, yb[sl].im, ri);
      ir = mfma(xa[sl].im, yb[sl].re, ir);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    kbe_c128 *d = dst + (q + 4 * r) * 16 + row;
    cd v{rr[r] + ii[r], ri[r] - ir[r]};
    if (!p.overwrite) v = v + ld(d);
    st(d, v);
  }
}

// ------------------------------------------------------------------------------------------
// Host side: chunking, workspace layout and launches.
// ------------------------------------------------------------------------------------------
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static int chunk_terms(int N, bool mfma) {
  if (mfma) return 256;
  const int E = N * N;
  return E >= 64 ? 256 : (E >= 16 ? 1024 : 4096);
}

// Add class cls with nout outputs whose term indices lie below tmax (skipped when empty).
static void plan_add(FusedPlan &pl, int cls, int nout, int tmax, int E, size_t &off) {
  if (nout <= 0 || tmax <= 0) return;
  const int k = pl.ncls++;
  pl.cls[k] = cls;
  pl.nout[k] = nout;
  pl.nchunk[k] = (tmax + pl.SC - 1) / pl.SC;
  pl.ngroup[k] = (nout + pl.MO - 1) / pl.MO;
  pl.off[k] = (int64_t)off;
  const int64_t wgs = (int64_t)pl.nchunk[k] * ((pl.ngroup[k] + 3) / 4);
  pl.first_wg[k + 1] = pl.first_wg[k] + (wgs + 7) / 8 * 8;
  off += al256(sizeof(kbe_c128) * (size_t)pl.nchunk[k] * nout * E);
}

static FusedPlan plan_init(int N, bool mfma) {
  FusedPlan pl{};
  pl.SC = chunk_terms(N, mfma);
  pl.MO = mfma ? 4 : 1;
  return pl;
}

static size_t plan_forward(int N, int ntau, int n, int m0, int m1, unsigned flags, bool mfma,
                           FusedPlan &pl) {
  pl = plan_init(N, mfma);
  const int E = N * N, M = m1 - m0;
  size_t off = 0;
  const bool th = ntau > 0;
  if (flags & KBE_OUT_IR) {
    plan_add(pl, C_IRC, M, m1, E, off);
    if (n > m0) plan_add(pl, C_IRR, M, n + 1, E, off);
  }
  if (flags & KBE_OUT_IL) plan_add(pl, C_IL, M, m1, E, off);
  if ((flags & KBE_OUT_ITV) && th) plan_add(pl, C_ITV, M, ntau, E, off);
  if ((flags & KBE_OUT_JTV) && th) {
    plan_add(pl, C_JR, ntau, n + 1, E, off);
    plan_add(pl, C_JM, ntau, ntau, E, off);
  }
  return off;
}

static size_t plan_adjoint(int N, int ntau, int n, int m0, int m1, unsigned flags, bool mfma,
                           FusedPlan &pl) {
  pl = plan_init(N, mfma);
  const int E = N * N;
  size_t off = 0;
  const bool th = ntau > 0, M = m1 > m0;
  const bool fITV = (flags & KBE_OUT_ITV) && th, fJTV = (flags & KBE_OUT_JTV) && th;
  if ((flags & KBE_OUT_IR) && M) {
    plan_add(pl, B_R1, n + 1, m1, E, off);
    plan_add(pl, B_R2, n + 1, m1, E, off);
  }
  if (fJTV) plan_add(pl, B_R3, n + 1, ntau, E, off);
  if ((flags & KBE_OUT_IL) && M) plan_add(pl, B_L, n + 1, m1, E, off);
  if (fITV && M) plan_add(pl, B_T1, ntau, m1, E, off);
  if (fJTV) {
    plan_add(pl, B_T2, ntau, ntau, E, off);
    plan_add(pl, G_MAT, ntau, ntau, E, off);
  }
  return off;
}

size_t collision_ws_bytes(int N, int nt, int ntau, int n, int m0, int m1, unsigned flags) {
  (void)nt;
  FusedPlan pl;
  const bool mfma = N == 16 && !(flags & KBE_FORCE_GENERIC);
  return plan_forward(N, ntau, n, m0, m1, flags, mfma, pl);
}

size_t collision_vjp_ws_bytes(int N, int nt, int ntau, int n, int m0, int m1, unsigned flags) {
  (void)nt;
  FusedPlan pl;
  const bool mfma = N == 16 && !(flags & KBE_FORCE_GENERIC);
  return plan_adjoint(N, ntau, n, m0, m1, flags, mfma, pl);
}

static void launch_fused(const Params &p, const FusedPlan &pl, bool mfma, char *ws,
                         hipStream_t st) {
  const int64_t wgs = pl.first_wg[pl.ncls];
  if (wgs == 0) return;
  const dim3 grid((unsigned)wgs), block(256);
  if (mfma) hipLaunchKernelGGL(stream_fused<true>, grid, block, 0, st, p, pl, ws);
  else hipLaunchKernelGGL(stream_fused<false>, grid, block, 0, st, p, pl, ws);
}

// Reduce the listed classes (those present in the plan) into out[nout][E].
static void reduce_into(const Params &p, const FusedPlan &pl, std::initializer_list<int> classes,
                        char *ws, int nout, kbe_c128 *out, bool accumulate, hipStream_t st) {
  RedIn in{};
  in.SC = pl.SC;
  for (int c : classes)
    for (int k = 0; k < pl.ncls; ++k)
      if (pl.cls[k] == c && in.nparts < 3) {
        in.a[in.nparts] = (const kbe_c128 *)(ws + pl.off[k]);
        in.cls[in.nparts] = c;
        in.nchunk[in.nparts] = pl.nchunk[k];
        ++in.nparts;
      }
  const int64_t nel = (int64_t)nout * p.N * p.N;
  if (nel == 0) return;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, st, p, in,
                     nout, out, accumulate ? 1 : 0);
}

hipError_t launch_collision(const Params &p, unsigned flags, kbe_c128 *IR, kbe_c128 *IL,
                            kbe_c128 *Itv, kbe_c128 *Jtv, void *ws, hipStream_t st) {
  const bool mfma = p.N == 16 && !(flags & KBE_FORCE_GENERIC);
  FusedPlan pl;
  plan_forward(p.N, p.ntau, p.n, p.m0, p.m1, flags, mfma, pl);
  char *w = (char *)ws;
  launch_fused(p, pl, mfma, w, st);
  const int M = p.m1 - p.m0;
  if (flags & KBE_OUT_IR) reduce_into(p, pl, {C_IRC, C_IRR}, w, M, IR, false, st);
  if (flags & KBE_OUT_IL) reduce_into(p, pl, {C_IL}, w, M, IL, false, st);
  if (flags & KBE_OUT_ITV) reduce_into(p, pl, {C_ITV}, w, M, Itv, false, st);
  if ((flags & KBE_OUT_JTV) && p.ntau > 0) reduce_into(p, pl, {C_JR, C_JM}, w, p.ntau, Jtv, false, st);
  return hipGetLastError();
}

hipError_t launch_collision_vjp(const Params &p, unsigned flags, kbe_c128 *gmat,
                                const kbe_sigma_row *gS, void *ws, hipStream_t st) {
  const bool mfma = p.N == 16 && !(flags & KBE_FORCE_GENERIC);
  FusedPlan pl;
  plan_adjoint(p.N, p.ntau, p.n, p.m0, p.m1, flags, mfma, pl);
  char *w = (char *)ws;
  launch_fused(p, pl, mfma, w, st);
  // self-energy gradients: overwritten
  reduce_into(p, pl, {B_R1, B_R2, B_R3}, w, p.n + 1, gS->ret, false, st);
  reduce_into(p, pl, {B_L}, w, p.n + 1, gS->les, false, st);
  if (p.ntau > 0) reduce_into(p, pl, {B_T1, B_T2}, w, p.ntau, gS->tv, false, st);
  // Green's-function gradients
  const int64_t n1 = p.n + 1;
  const int64_t nblk = n1 * n1 + n1 + (p.ntau > 0 ? n1 * p.ntau : 0);
  if (mfma) {
    hipLaunchKernelGGL(grad_mfma16, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, st, p, nblk);
  } else {
    const int64_t th = nblk * p.N * p.N;
    hipLaunchKernelGGL(grad_generic, dim3((unsigned)((th + 255) / 256)), dim3(256), 0, st, p, nblk);
  }
  if (p.fJTV) reduce_into(p, pl, {G_MAT}, w, p.ntau, gmat, !p.overwrite, st);
  return hipGetLastError();
}

}  // namespace kbe
