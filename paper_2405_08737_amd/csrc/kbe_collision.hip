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
// partial sums of MO consecutive outputs over one chunk (on the MFMA path a workgroup of 4 waves
// x MO = 2 outputs shares each staged Q block between 8 P blocks) and writes them to the
// workspace; a reduce kernel adds the chunks
// of every output in a fixed order, so results are deterministic (no floating-point atomics).
// Workgroups are laid out chunk-fastest and every class starts on a multiple of 8 workgroups:
// with round-robin dispatch over the 8 XCDs, all tasks of a chunk land on one XCD and its L2
// holds that chunk's Q blocks.
//
// Implementations of a task:
//   * wg_task_mfma16 (N = 16): FP64 matrix cores (v_mfma_f64_4x4x4, layout below), three real
//     products per complex one (three accumulators per output); Q staged in LDS per term,
//     the streamed blocks prefetched into registers a term ahead.
//   * wg_task_small (N <= 8): vector ALU; a wave holds 64 / N^2 streamed blocks side by side,
//     each lane one element of a block and its share of every output row (the sum over that
//     element's index taken once per task through LDS); Q staged in LDS in batches of terms.
//   * task_generic (any N <= 16): vector ALU, one output per wave, one output element per lane,
//     several terms per wave for small N summed across lanes at the end.
// On the MFMA path a class can carry a second one on its tasks (FusedPlan::pair): the greater
// form's C_GRU beside C_IL / C_ILX and B_GRU beside B_L read the same streamed blocks into the
// same outputs, each with its own Q, weights, accumulators and partials.
#include <map>
#include <mutex>
#include <tuple>
#include "kbe_dev.h"
#include "kbe_internal.h"

#include <initializer_list>
#include <utility>

namespace kbe {

enum Cls {
  C_IRC,   // I^R, s <= m:  w[n][s] Sigma^R(s) kp[s][m]               (G^<(s,m) stored)
  C_IRR,   // I^R, s > m : -w[n][s] Sigma^R(s) kp[m][s]^dagger        (G^<(s,m) = -kp[m][s]^dag)
  C_IL,    // I^<, s <= m:  w[m][s] Sigma^<(s) G^R(m,s)^dagger
  C_ITV,   // I^]:  -i wtau[j] Sigma^](j) tv[m][J-j]^dagger
  C_JR,    // J^] real-time part:  w[n][s] Sigma^R(s) tv[s][j]
  C_JM1,   // J^] Matsubara part on [0, tau_j]:   -wf[j][l] Sigma^](l) G^M(beta + tau_l - tau_j)
  C_JM2,   // J^] Matsubara part on [tau_j, beta]: wb[j][l] Sigma^](l) G^M(tau_l - tau_j)
  B_R1,    // adjoint: gSigma^R(s) from C_IRC terms
  B_R2,    // adjoint: gSigma^R(s) from C_IRR terms
  B_R3,    // adjoint: gSigma^R(s) from C_JR terms
  B_L,     // adjoint: gSigma^<(s) from C_IL terms
  B_T1,    // adjoint: gSigma^](j) from C_ITV terms
  B_T2A,   // adjoint: gSigma^](l) from C_JM1 terms
  B_T2B,   // adjoint: gSigma^](l) from C_JM2 terms
  G_MAT1,  // adjoint: gG^M(k) from C_JM1 terms
  G_MAT2,  // adjoint: gG^M(k) from C_JM2 terms
  // the greater form (KBE_GREATER): G^>(s,m) = G^<(s,m) + D(s,m) in I^R, with D(s,m) = G^R(s,m)
  // for s > m, G^R(m,m) at s = m and -G^R(m,s)^dagger for s < m; in I^<, C_IL reads a
  // Sigma^> = Sigma^R + Sigma^< row formed once in the workspace
  C_GRL,   // I^R, s > m :  w[n][s] Sigma^R(s) kp[s][m]
  C_GRD,   // I^R, s = m :  w[n][m] Sigma^R(m) rdiag[m]
  C_GRU,   // I^R, s < m : -w[n][s] Sigma^R(s) kp[m][s]^dagger
  // adjoint of the greater form: gSigma^R(s) from the D parts of C_GRL, C_GRD, C_GRU
  B_GRL,   // s > m:  w[n][s] gIR(m) kp[s][m]^dagger
  B_GRD,   // s = m:  w[n][s] gIR(s) rdiag[s]^dagger
  B_GRU,   // s < m: -w[n][s] gIR(m) kp[m][s]
  // both forms in one call (the propagations): I^< of the greater form reads the Sigma^> row
  // through its own class, beside C_IL on the Sigma^< row
  C_ILX,   // I^<, s <= m:  w[m][s] Sigma^>(s) G^R(m,s)^dagger
  // the greater form's extra adjoint terms when gIR and gIL are one array (KBE_INT_SAMECOT):
  // B_L and B_GRU on their shared blocks kp[m][s], m > s, with weight w[m][s] - w[n][s]
  B_LGU,   // m >= s: (w[m][s] - [m > s] w[n][s]) gIL(m) G^R(m,s)  (G^R(s,s) = rdiag[s])
  NCLS
};
enum Op { OP_N = 0, OP_H = 1, OP_HN = 2 };

template <int CLS>
__host__ __device__ constexpr int cls_op() {
  return (CLS == C_IRR || CLS == C_IL || CLS == C_ILX || CLS == C_ITV || CLS == B_R1 || CLS == B_R3 ||
          CLS == B_T2A || CLS == B_T2B || CLS == C_GRU || CLS == B_GRL ||
          CLS == B_GRD)
             ? OP_H
             : ((CLS == G_MAT1 || CLS == G_MAT2) ? OP_HN : OP_N);
}

// Term-index range [lo, hi) of output o.  Empty ranges too stay inside the indices for which the
// class's shared operand exists: the workgroup tasks stage that operand for every term of the
// union of their outputs' ranges.
template <int CLS>
__host__ __device__ __forceinline__ void cls_range(const Params &p, int o, int &lo, int &hi) {
  const int m = p.m0 + o;
  switch (CLS) {
    case C_IRC: lo = 0; hi = m + 1; break;
    case C_IRR: lo = m + 1; hi = p.n + 1; break;
    case C_IL: case C_ILX: lo = 0; hi = m + 1; break;
    case C_GRL: lo = m + 1; hi = p.n + 1; break;
    case C_GRD: lo = m; hi = m + 1; break;
    case C_GRU: lo = 0; hi = m; break;
    case C_ITV: lo = 0; hi = p.ntau; break;
    case C_JR: lo = 0; hi = p.n + 1; break;
    case C_JM1: lo = 0; hi = o + 1; break;        // l <= j
    case C_JM2: lo = o; hi = p.ntau; break;       // l >= j
    case B_R1: lo = o > p.m0 ? o : p.m0; hi = p.m1; break;
    case B_R2: lo = p.m0; hi = o < p.m1 ? o : p.m1; break;
    case B_R3: lo = 0; hi = p.ntau; break;
    case B_L: case B_LGU: lo = o > p.m0 ? o : p.m0; hi = p.m1; break;
    case B_T1: lo = p.m0; hi = p.m1; break;
    case B_T2A: lo = o; hi = p.ntau; break;       // output l, terms j >= l
    case B_T2B: lo = 0; hi = o + 1; break;        // output l, terms j <= l
    case G_MAT1: lo = 0; hi = o + 1; break;       // output k, terms l <= k
    case G_MAT2: lo = o; hi = p.ntau; break;      // output k, terms l >= k
    case B_GRL: lo = p.m0; hi = o < p.m1 ? o : p.m1; break;            // terms m < s
    case B_GRD:  // m = s; an empty range stays inside [m0, m1), where the shared operand exists
      lo = (o >= p.m0 && o < p.m1) ? o : p.m0;
      hi = (o >= p.m0 && o < p.m1) ? o + 1 : p.m0;
      break;
    case B_GRU: lo = o + 1 > p.m0 ? o + 1 : p.m0; hi = p.m1; break;     // terms m > s
  }
}

// Shared operand of term t.
template <int CLS>
__host__ __device__ __forceinline__ const kbe_c128 *cls_Q(const Params &p, int t) {
  const int64_t E = bsz(p);
  switch (CLS) {
    case C_IRC: case C_IRR: case C_JR: case C_GRL: case C_GRD: case C_GRU:
      return p.ret + t * E;
    case C_IL: return p.les + t * E;
    case C_ILX: return p.sgt + t * E;
    case C_ITV: case C_JM1: case C_JM2: case G_MAT1: case G_MAT2: return p.stv + t * E;
    case B_R1: case B_R2: case B_GRL: case B_GRD: case B_GRU: return p.gIR + (t - p.m0) * E;
    case B_L: case B_LGU: return p.gIL + (t - p.m0) * E;
    case B_T1: return p.gItv + (t - p.m0) * E;
    case B_R3: case B_T2A: case B_T2B: return p.gJ + t * E;
  }
  return nullptr;
}

// Every term weight is a real quadrature weight times a class constant f in {1, -1, i, -i}.
template <int CLS>
__host__ __device__ constexpr int cls_fre() {
  return (CLS == C_IRR || CLS == C_JM1 || CLS == B_R2 || CLS == B_T2A || CLS == G_MAT1 ||
          CLS == C_GRU || CLS == B_GRU)
             ? -1
         : (CLS == C_ITV || CLS == B_T1)                                                 ? 0
                                                                                         : 1;
}
template <int CLS>
__host__ __device__ constexpr int cls_fim() {
  return CLS == C_ITV ? -1 : (CLS == B_T1 ? 1 : 0);
}

// Addresses of the real weight (the term weight is f w) and of the streamed block P of term t of
// output o.  Only address arithmetic: they are valid to read when t lies in o's range.
template <int CLS>
__host__ __device__ __forceinline__ void cls_wpP(const Params &p, int o, int t, const double *&w,
                                                 const kbe_c128 *&P) {
  const int64_t E = bsz(p);
  const int J = p.J, m = p.m0 + o;
  switch (CLS) {
    case C_IRC: w = p.w + ((int64_t)p.n * p.nt + t); P = kp_blk(p, t, m); break;
    case C_IRR: w = p.w + ((int64_t)p.n * p.nt + t); P = kp_blk(p, m, t); break;
    case C_IL: case C_ILX:
      w = p.w + ((int64_t)m * p.nt + t);
      P = t < m ? kp_blk(p, m, t) : p.rdiag + m * E;
      break;
    case C_ITV: w = p.wtau + t; P = tv_blk(p, m, J - t); break;
    case C_GRL: w = p.w + ((int64_t)p.n * p.nt + t); P = kp_blk(p, t, m); break;
    case C_GRD: w = p.w + ((int64_t)p.n * p.nt + t); P = p.rdiag + m * E; break;
    case C_GRU: w = p.w + ((int64_t)p.n * p.nt + t); P = kp_blk(p, m, t); break;
    case C_JR: w = p.w + ((int64_t)p.n * p.nt + t); P = tv_blk(p, t, o); break;
    case C_JM1:  // l = t <= j = o
      w = p.wf + ((int64_t)o * p.ntau + t);
      P = p.mat + (J + t - o) * E;
      break;
    case C_JM2:  // l = t >= j = o; the rule over [tau_j, beta] is the mirrored forward rule
      w = p.wf + ((int64_t)(J - o) * p.ntau + (J - t));
      P = p.mat + (t - o) * E;
      break;
    case B_R1: w = p.w + ((int64_t)p.n * p.nt + o); P = kp_blk(p, o, t); break;
    case B_R2: w = p.w + ((int64_t)p.n * p.nt + o); P = kp_blk(p, t, o); break;
    case B_R3: w = p.w + ((int64_t)p.n * p.nt + o); P = tv_blk(p, o, t); break;
    case B_GRL: w = p.w + ((int64_t)p.n * p.nt + o); P = kp_blk(p, o, t); break;
    case B_GRD: w = p.w + ((int64_t)p.n * p.nt + o); P = p.rdiag + o * E; break;
    case B_GRU: w = p.w + ((int64_t)p.n * p.nt + o); P = kp_blk(p, t, o); break;
    case B_L: case B_LGU:
      w = p.w + ((int64_t)t * p.nt + o);
      P = t > o ? kp_blk(p, t, o) : p.rdiag + o * E;
      break;
    case B_T1: w = p.wtau + o; P = tv_blk(p, t, J - o); break;
    case B_T2A:  // j = t >= l = o
      w = p.wf + ((int64_t)t * p.ntau + o);
      P = p.mat + (J + o - t) * E;
      break;
    case B_T2B:  // j = t <= l = o
      w = p.wf + ((int64_t)(J - t) * p.ntau + (J - o));
      P = p.mat + (o - t) * E;
      break;
    case G_MAT1: {  // l = t <= k = o, j = l + J - k
      const int j = t + J - o;
      w = p.wf + ((int64_t)j * p.ntau + t);
      P = p.gJ + j * E;
      break;
    }
    case G_MAT2: {  // l = t >= k = o, j = l - k
      const int j = t - o;
      w = p.wf + ((int64_t)(J - j) * p.ntau + (J - t));
      P = p.gJ + j * E;
      break;
    }
  }
}

// The weight a term subtracts from the one cls_wpP addresses (B_LGU below the diagonal: B_GRU's
// w[n][s]); 0 for every other class.  Read only for a term inside its output's range.
template <int CLS>
__device__ __forceinline__ double cls_w2(const Params &p, int o, int t) {
  if constexpr (CLS == B_LGU) return t > o ? p.w[(int64_t)p.n * p.nt + o] : 0.0;
  else return 0.0;
}

template <int CLS>
__device__ __forceinline__ void cls_wP(const Params &p, int o, int t, double &w,
                                       const kbe_c128 *&P) {
  const double *wp;
  cls_wpP<CLS>(p, o, t, wp, P);
  w = *wp;
  if constexpr (CLS == B_LGU) w -= cls_w2<CLS>(p, o, t);
}

// Complex weight c = f w and block P of term t of output o.
template <int CLS>
__device__ __forceinline__ void cls_P(const Params &p, int o, int t, cd &c, const kbe_c128 *&P) {
  double w;
  cls_wP<CLS>(p, o, t, w, P);
  c = {cls_fre<CLS>() * w, cls_fim<CLS>() * w};
}

__device__ __forceinline__ void range_rt(int cls, const Params &p, int o, int &lo, int &hi) {
  switch (cls) {
#define KBE_CASE(C) \
  case C: cls_range<C>(p, o, lo, hi); break;
    KBE_CASE(C_IRC) KBE_CASE(C_IRR) KBE_CASE(C_IL) KBE_CASE(C_ITV) KBE_CASE(C_JR) KBE_CASE(C_JM1)
    KBE_CASE(C_JM2) KBE_CASE(B_R1) KBE_CASE(B_R2) KBE_CASE(B_R3) KBE_CASE(B_L) KBE_CASE(B_T1)
    KBE_CASE(B_T2A) KBE_CASE(B_T2B) KBE_CASE(G_MAT1) KBE_CASE(G_MAT2) KBE_CASE(C_GRL)
    KBE_CASE(C_GRD) KBE_CASE(C_GRU) KBE_CASE(B_GRL) KBE_CASE(B_GRD)
    KBE_CASE(B_GRU) KBE_CASE(C_ILX) KBE_CASE(B_LGU)
#undef KBE_CASE
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
      cd c;
      const kbe_c128 *P;
      cls_P<CLS>(p, o, t, c, P);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r >= R) break;
        const int e = E <= 64 ? lane % E : lane + 64 * r;
        if (e >= E) break;
        const int i = e / N, j = e % N;
        cd s = czero();
        for (int k = 0; k < N; ++k) {
          if (OP == OP_N) s = s + ld(Q + i * N + k) * ld(P + k * N + j);
          else if (OP == OP_H) s = s + ld(Q + i * N + k) * cj(ld(P + j * N + k));
          else s = s + cj(ld(Q + k * N + i)) * ld(P + k * N + j);
        }
        acc[r] = acc[r] + c * s;
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
// Small-block task (N <= 8): vector ALU, workgroup-tiled like the MFMA task.
//
// A wave holds GS = 64 / (N*N) blocks side by side ("slots", lane = slot * N*N + element) and
// every slot carries ML outputs, so a wave covers MO = GS * ML consecutive outputs and one load
// instruction streams GS blocks.  Lane (a, b) of a slot holds element (a, b) of its outputs'
// streamed blocks and accumulates that element's share of every output row i (a k-split):
//   OP_N : element (k, j) of P adds Q[i][k] c P[k][j]           to out[i][j]
//   OP_H : element (j, k) of P adds Q[i][k] c conj(P[j][k])     to out[i][j]
//   OP_HN: element (k, j) of P adds conj(Q[k][i]) c P[k][j]      to out[i][j]
// so the lane reads one column of Q (one row for OP_HN) per term, from an LDS copy shared by
// the workgroup (staged TB terms at a time, double-buffered, one barrier per TB terms), and
// the streamed blocks of the next term are in flight while a term is computed.  The sum over
// k is taken once per task, through LDS, in a fixed order.
// ------------------------------------------------------------------------------------------
template <int N>
struct SmallCfg {
  static constexpr int E = N * N;
  static constexpr int GS = 64 / E;                         // slots per wave
  static constexpr int ML = N >= 3 ? 4 : (N == 2 ? 2 : 1);  // outputs per slot
  static constexpr int MO = GS * ML;                        // outputs per wave
  static constexpr int TB = 256 / E;                        // terms per staged Q batch
  static constexpr int LQ = N == 1 ? 1 : N + 1;             // LDS row stride (complex)
  static constexpr int QB = TB * N * LQ;                    // complex numbers per batch
  static constexpr int RS = 65;                             // reduction row stride (complex)
  static constexpr int RED = 4 * N * RS;                    // reduction scratch, 4 waves
  static constexpr int LDS = 2 * QB > RED ? 2 * QB : RED;
};

template <int N, int CLS>
__device__ __forceinline__ void wg_task_small(const Params &p, int nout, int ngroup, int ch,
                                              int gb, int SC, kbe_c128 *base, cd *smem,
                                              int *rng) {
  using C = SmallCfg<N>;
  constexpr int E = C::E, GS = C::GS, ML = C::ML, MO = C::MO, TB = C::TB, LQ = C::LQ;
  constexpr int OP = cls_op<CLS>();
  constexpr int FR = cls_fre<CLS>(), FI = cls_fim<CLS>();  // term weight c = (FR + i FI) w
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = gb * 4 + wave;
  const int o0 = g * MO;
  // lane -> (slot, element); the lanes past GS*E (N = 3, 5, 6, 7) are idle: they read a valid
  // element and store nothing
  const bool act = lane < GS * E;
  const int slot = GS == 1 ? 0 : (act ? lane / E : 0);
  const int e = act ? lane - slot * E : 0;
  const int a = e / N, b = e - (e / N) * N;
  int lo[ML], hi[ML];
  bool val[ML];
#pragma unroll
  for (int u = 0; u < ML; ++u) {
    const int o = o0 + slot * ML + u;
    val[u] = act && g < ngroup && o < nout;
    lo[u] = hi[u] = 0;
    if (val[u]) cls_range<CLS>(p, o, lo[u], hi[u]);
  }
  // workgroup union of the term ranges (wave-uniform loop over the wave's outputs)
  int wlo = 1 << 30, whi = 0;
  if (g < ngroup) {
    for (int v = 0; v < MO; ++v) {
      if (o0 + v >= nout) break;
      int l, h;
      cls_range<CLS>(p, o0 + v, l, h);
      wlo = l < wlo ? l : wlo;
      whi = h > whi ? h : whi;
    }
  }
  if (lane == 0) {
    rng[2 * wave] = wlo;
    rng[2 * wave + 1] = whi;
  }
  lds_barrier();
  int T0 = 1 << 30, T1 = 0;
  for (int w = 0; w < 4; ++w) {
    T0 = rng[2 * w] < T0 ? rng[2 * w] : T0;
    T1 = rng[2 * w + 1] > T1 ? rng[2 * w + 1] : T1;
  }
  T0 = __builtin_amdgcn_readfirstlane(T0 > ch * SC ? T0 : ch * SC);
  T1 = __builtin_amdgcn_readfirstlane(T1 < (ch + 1) * SC ? T1 : (ch + 1) * SC);
  cd acc[ML][N];
#pragma unroll
  for (int u = 0; u < ML; ++u)
#pragma unroll
    for (int i = 0; i < N; ++i) acc[u][i] = czero();
  if (T0 < T1) {
    // staging: thread tid < TB*E copies element r = (qi, qk) of Q(T + tq)
    const bool stager = tid < TB * E;
    const int tq = stager ? tid / E : 0, r = tid - tq * E;
    const int qi = r / N, qk = r - (r / N) * N;
    const int qdst = tq * N * LQ + (OP == OP_HN ? qi * LQ + qk : qk * LQ + qi);
    auto stage_ld = [&](int T) -> cd {
      int t = T + tq;
      t = t < T1 ? t : T1 - 1;
      return ld(cls_Q<CLS>(p, t) + r);
    };
    // The loads are unconditional (an output without term t reads a valid dummy and gets
    // weight 0), so the number of loads in flight is fixed and the wait for term t does not
    // wait for the prefetches of term t + 1.
    // The weight of an absent term is zeroed when the term is computed, not here, so that
    // nothing waits for a prefetch before its use.
    struct Term {
      double w[ML], w2[ML];  // w2: the weight subtracted (cls_w2; B_LGU only)
      bool in[ML];
      cd x[ML];
    };
    auto setup = [&](int t, Term &tm) {
#pragma unroll
      for (int u = 0; u < ML; ++u) {
        const double *wp;
        const kbe_c128 *P;
        cls_wpP<CLS>(p, o0 + slot * ML + u, t, wp, P);
        tm.in[u] = t >= lo[u] && t < hi[u];
        wp = tm.in[u] ? wp : p.w;
        P = tm.in[u] ? P : p.rdiag;
        tm.w[u] = *wp;
        if constexpr (CLS == B_LGU) tm.w2[u] = tm.in[u] ? cls_w2<CLS>(p, o0 + slot * ML + u, t) : 0.0;
        tm.x[u] = ld(P + e);
      }
    };
    const int R = OP == OP_H ? b : a;
    auto compute = [&](const cd *qs, const Term &tm) {
      cd y[ML];
#pragma unroll
      for (int u = 0; u < ML; ++u) {
        const cd xx = OP == OP_H ? cj(tm.x[u]) : tm.x[u];
        double wu = tm.in[u] ? tm.w[u] : 0.0;
        if constexpr (CLS == B_LGU) wu -= tm.w2[u];
        if (FI == 0) y[u] = (FR * wu) * xx;
        else y[u] = cd{-(FI * wu) * xx.im, (FI * wu) * xx.re};
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const cd q = qs[R * LQ + i];
        const double qi = OP == OP_HN ? -q.im : q.im;
#pragma unroll
        for (int u = 0; u < ML; ++u) {  // four fused multiply-adds per complex one
          acc[u][i].re = __builtin_fma(q.re, y[u].re, acc[u][i].re);
          acc[u][i].re = __builtin_fma(-qi, y[u].im, acc[u][i].re);
          acc[u][i].im = __builtin_fma(q.re, y[u].im, acc[u][i].im);
          acc[u][i].im = __builtin_fma(qi, y[u].re, acc[u][i].im);
        }
      }
    };
    // Batch b of Q (terms T0 + b TB ...) lives in staging buffer b % 2: written at the start of
    // batch b (loaded a batch earlier), then one barrier.  Terms ping-pong between two
    // register sets, so no prefetched value is copied (a copy would wait for its load).
    Term A, B;
    cd qn;
    if (stager) smem[qdst] = stage_ld(T0);
    setup(T0, A);
    if (stager) qn = stage_ld(T0 + TB);
    lds_barrier();
    auto step = [&](int t, const Term &cu, Term &nx) {
      const int rel = t - T0, bt = rel / TB, tt = rel - bt * TB;
      if (tt == 0 && rel > 0) {  // uniform: a new batch starts at term t
        if (stager) smem[(bt & 1) * C::QB + qdst] = qn;
        lds_barrier();
        if (stager) qn = stage_ld(t + TB);
      }
      setup(t + 1 < T1 ? t + 1 : t, nx);  // next term, in flight during compute
      // keep the loads of term t + 1 after those of term t (the load counter retires in order)
      __builtin_amdgcn_sched_barrier(0);
      compute(smem + (bt & 1) * C::QB + tt * N * LQ, cu);
      __builtin_amdgcn_sched_barrier(0);
    };
    for (int t = T0; t < T1; t += 2) {
      step(t, A, B);
      if (t + 1 >= T1) break;
      step(t + 1, B, A);
    }
    lds_barrier();  // the reduction below reuses the staging buffers
  }
  // sum over k: rows of red are output rows i, columns are lanes
  cd *red = smem + wave * N * C::RS;
  const int oi = e / N, oj = e - (e / N) * N;  // this lane's output element (oi, oj)
#pragma unroll
  for (int u = 0; u < ML; ++u) {
#pragma unroll
    for (int i = 0; i < N; ++i) red[i * C::RS + lane] = acc[u][i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool has = val[u] && hi[u] > ch * SC && lo[u] < (ch + 1) * SC;
    cd s = czero();
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int src = slot * E + (OP == OP_H ? oj * N + k : k * N + oj);
      s = s + red[oi * C::RS + src];
    }
    if (has) st(base + ((int64_t)ch * nout + o0 + slot * ML + u) * E + e, s);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ------------------------------------------------------------------------------------------
// FP64 MFMA task (N = 16): outputs o0..o0+no-1 (no <= MO), terms t in [t0, t1).
//
// Matrix cores: v_mfma_f64_4x4x4 (four independent 4x4x4 blocks per instruction; on gfx950 it
// sustains about 1.5x the FP64 rate of the 16x16x4 form).  Lane layout (checked with an
// in-bounds probe on gfx950): A[b][i][k] at lane 4b+i+16k, B[b][k][j] at lane 4b+j+16k,
// D[b][i][j] at lane 4b+j+16i.  A 16x16x16 product D = A B is cut into tile rows ti and
// k-chunks kc (4 each); one instruction computes the four tiles (ti, tj = b) of a tile row:
//   lane l supplies A[4ti + l%4][4kc + l/16] (a 4x4 tile, the same for every b) and
//   B[4kc + l/16][l%16] (rows 4kc..4kc+3 of B: a contiguous 1 KiB slab of a row-major block),
// and accumulator ti of lane l holds D[4ti + l/16][l%16].
//
// The small operand Q is always A and the streamed block is always B, so the streamed block is
// read as whole slabs (OP_N, OP_HN) or as 64-byte row segments (OP_H, which needs its columns):
//   OP_N : A = Q,       B = P'
//   OP_H : A = Q,       B = P'^dagger,  P' = conj(c) P   (then Q P'^dag = c Q P^dag)
//   OP_HN: A = Q^dagger, B = P'
// with P' = c P for OP_N and OP_HN.  Each complex product is three real ones (see
// term_compute); the sums of Q's parts are formed once per term and shared by all outputs.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// Workgroup task on the MFMA path: the 4 waves of a workgroup handle 4 groups of MO = 2
// consecutive outputs over the same chunk of terms, so they share every Q block.  Each term's
// Q block is staged once per workgroup in LDS (double-buffered, rows padded to 20 complex
// numbers so the 4x4 A-tile reads are free of bank conflicts) while every wave prefetches its
// outputs' streamed slabs for the next term into registers; one barrier per term.
constexpr int MO_MFMA = 2;
constexpr int QLD = 20;  // LDS row stride of a staged 16x16 block, in complex numbers

template <int MO>
struct TermOps {
  const kbe_c128 *P[MO];
  double w[MO];  // real weight; 0 when the output has no such term
};

template <int MO>
struct TermP {
  cd v[4][MO];  // slab value for k-chunk kc of output u
};

// Weights and block addresses of term t for the wave's outputs.  Everything here is wave-uniform
// (scalar control flow); an output without this term gets weight 0 and a valid dummy block,
// so loads and products below run unconditionally.  Nothing is computed from the loaded weights
// here: they are prefetches, first used by term_compute one term later.
template <int CLS, int MO>
__device__ __forceinline__ void term_setup(const Params &p, int o0, int t, const int *lo,
                                           const int *hi, int no, TermOps<MO> &ts) {
#pragma unroll
  for (int u = 0; u < MO; ++u) {
    ts.w[u] = 0.0;
    ts.P[u] = p.rdiag;
    if (u < no && t >= lo[u] && t < hi[u]) cls_wP<CLS>(p, o0 + u, t, ts.w[u], ts.P[u]);
  }
}

template <int CLS, int MO>
__device__ __forceinline__ void term_loadP(const TermOps<MO> &ts, int lk, int lc, TermP<MO> &tp) {
  constexpr int OP = cls_op<CLS>();
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const int pidx = OP == OP_H ? lc * 16 + 4 * kc + lk : (4 * kc + lk) * 16 + lc;
#pragma unroll
    for (int u = 0; u < MO; ++u) tp.v[kc][u] = ld(ts.P[u] + pidx);
  }
}

// MFMA with the A operand negated (the f64 forms take negate modifiers).
__device__ __forceinline__ double mfma4na(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 1);
}

// Matrix-core work of one term for the wave's outputs; Q is read from the LDS tile qs.
template <int CLS, int MO>
__device__ __forceinline__ void term_compute(const TermOps<MO> &ts, const TermP<MO> &tp,
                                             const cd *qs, int lr, int lk, double (&k1)[MO][4],
                                             double (&k2)[MO][4], double (&k3)[MO][4]) {
  constexpr int OP = cls_op<CLS>();
  // B scale: c for OP_N / OP_HN, conj(c) for OP_H, with c = f w, f in {1, -1, i, -i}
  constexpr int FR = cls_fre<CLS>(), FI = OP == OP_H ? -cls_fim<CLS>() : cls_fim<CLS>();
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    // operands a = (ar, sa ai), b = (br, sb bi): sa = -1 for OP_HN (A = Q^dag), sb = -1 for
    // OP_H (B = P^dag); the product takes three real MFMA products (Gauss):
    //   k1 += (ar + sa ai) br,  k2 += ar (sb bi - br),  k3 += (sa ai) (br + sb bi),
    //   Re = k1 - k3, Im = k1 + k2.
    double ar[4], ai[4], as[4];
#pragma unroll
    for (int ti = 0; ti < 4; ++ti) {
      const cd v = OP == OP_HN ? qs[(4 * kc + lk) * QLD + 4 * ti + lr]
                               : qs[(4 * ti + lr) * QLD + 4 * kc + lk];
      ar[ti] = v.re;
      ai[ti] = v.im;
      as[ti] = OP == OP_HN ? v.re - v.im : v.re + v.im;
    }
    double br[MO], bd[MO], bp[MO];
#pragma unroll
    for (int u = 0; u < MO; ++u) {
      const cd x = tp.v[kc][u];
      cd pv;
      if (FI == 0) {
        const double s = FR * ts.w[u];
        pv = {s * x.re, s * x.im};
      } else {  // (FI i) w x
        const double s = FI * ts.w[u];
        pv = {-s * x.im, s * x.re};
      }
      const double bi = OP == OP_H ? -pv.im : pv.im;
      br[u] = pv.re;
      bd[u] = bi - pv.re;
      bp[u] = pv.re + bi;
    }
    // three passes over (output, tile row): an accumulator's updates are 4*MO instructions apart
#pragma unroll
    for (int pass = 0; pass < 3; ++pass) {
#pragma unroll
      for (int u = 0; u < MO; ++u) {
#pragma unroll
        for (int ti = 0; ti < 4; ++ti) {
          if (pass == 0) k1[u][ti] = mfma4(as[ti], br[u], k1[u][ti]);
          if (pass == 1) k2[u][ti] = mfma4(ar[ti], bd[u], k2[u][ti]);
          if (pass == 2) {
            if (OP == OP_HN) k3[u][ti] = mfma4na(ai[ti], bp[u], k3[u][ti]);
            else k3[u][ti] = mfma4(ai[ti], bp[u], k3[u][ti]);
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// One workgroup = chunk ch x output groups 4*gb .. 4*gb+3.  qbuf: 4 x 16 x QLD complex in LDS.
// All 256 threads reach every barrier: the term range is uniform over the workgroup.  The
// barriers order LDS only, so the global prefetches of the next term stay in flight across
// them.  CB >= 0: the tasks also compute class CB, whose terms are a subset of CLS's with the
// same streamed block and operation (C_GRU beside C_IL / C_ILX, B_GRU beside B_L): its Q staged
// beside CLS's (qbuf + 32 QLD), its own weights and accumulators, its partials into baseB.
template <int CLS, int CB = -1>
__device__ __forceinline__ void wg_task_mfma16(const Params &p, int nout, int ngroup, int ch,
                                               int gb, int SC, kbe_c128 *base, cd *qbuf,
                                               int *rng, kbe_c128 *baseB = nullptr) {
  constexpr int MO = MO_MFMA;
  constexpr bool DUAL = CB >= 0;
  constexpr int CB_ = DUAL ? CB : CLS;
  static_assert(!DUAL || cls_op<CB_>() == cls_op<CLS>(), "paired classes share the operation");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 3, lk = lane >> 4, lc = lane & 15;
  const int g = gb * 4 + wave;
  const int o0 = g * MO;
  const int no = g < ngroup ? (nout - o0 < MO ? nout - o0 : MO) : 0;
  int lo[MO], hi[MO], lob[MO], hib[MO];
  int wlo = 1 << 30, whi = 0;
#pragma unroll
  for (int u = 0; u < MO; ++u) {
    lo[u] = 0;
    hi[u] = 0;
    lob[u] = 0;
    hib[u] = 0;
    if (u < no) {
      cls_range<CLS>(p, o0 + u, lo[u], hi[u]);
      wlo = lo[u] < wlo ? lo[u] : wlo;
      whi = hi[u] > whi ? hi[u] : whi;
      if constexpr (DUAL) cls_range<CB_>(p, o0 + u, lob[u], hib[u]);  // inside [lo, hi)
    }
  }
  // workgroup union of the term ranges, clipped to the chunk
  if (lane == 0) {
    rng[2 * wave] = wlo;
    rng[2 * wave + 1] = whi;
  }
  lds_barrier();
  int T0 = 1 << 30, T1 = 0;
  for (int w = 0; w < 4; ++w) {
    T0 = rng[2 * w] < T0 ? rng[2 * w] : T0;
    T1 = rng[2 * w + 1] > T1 ? rng[2 * w + 1] : T1;
  }
  T0 = __builtin_amdgcn_readfirstlane(T0 > ch * SC ? T0 : ch * SC);
  T1 = __builtin_amdgcn_readfirstlane(T1 < (ch + 1) * SC ? T1 : (ch + 1) * SC);
  double k1[MO][4], k2[MO][4], k3[MO][4];
  double b1[MO][4], b2[MO][4], b3[MO][4];  // CB's accumulators
#pragma unroll
  for (int u = 0; u < MO; ++u)
#pragma unroll
    for (int ti = 0; ti < 4; ++ti) {
      k1[u][ti] = k2[u][ti] = k3[u][ti] = 0.0;
      b1[u][ti] = b2[u][ti] = b3[u][ti] = 0.0;
    }
  cd *const qb = qbuf + 32 * QLD;  // CB's Q buffers
  if (T0 < T1) {
    const int qrow = tid >> 4, qcol = tid & 15;  // this thread stages element (qrow, qcol)
    TermOps<MO> ta, tb, wa, wb;  // wa, wb: CB's weights (its blocks are CLS's)
    TermP<MO> pa, pb;
    // prologue: Q(T0) into buffer 0, slabs of T0 into pa
    qbuf[qrow * QLD + qcol] = ld(cls_Q<CLS>(p, T0) + tid);
    if constexpr (DUAL) qb[qrow * QLD + qcol] = ld(cls_Q<CB_>(p, T0) + tid);
    term_setup<CLS, MO>(p, o0, T0, lo, hi, no, ta);
    if constexpr (DUAL) term_setup<CB_, MO>(p, o0, T0, lob, hib, no, wa);
    term_loadP<CLS, MO>(ta, lk, lc, pa);
    for (int t = T0; t < T1; t += 2) {
      // even term t: compute from (ta, pa, buffer 0); prefetch t+1 into (tb, pb, buffer 1).
      // The prefetch is unconditional: past the range it re-reads the last term (unused).
      const int t1 = t + 1 < T1 ? t + 1 : T1 - 1;
      cd qn = ld(cls_Q<CLS>(p, t1) + tid), qnb;
      if constexpr (DUAL) qnb = ld(cls_Q<CB_>(p, t1) + tid);
      term_setup<CLS, MO>(p, o0, t1, lo, hi, no, tb);
      if constexpr (DUAL) term_setup<CB_, MO>(p, o0, t1, lob, hib, no, wb);
      term_loadP<CLS, MO>(tb, lk, lc, pb);
      lds_barrier();
      __builtin_amdgcn_sched_barrier(0);
      term_compute<CLS, MO>(ta, pa, qbuf, lr, lk, k1, k2, k3);
      if constexpr (DUAL) term_compute<CB_, MO>(wa, pa, qb, lr, lk, b1, b2, b3);
      qbuf[16 * QLD + qrow * QLD + qcol] = qn;
      if constexpr (DUAL) qb[16 * QLD + qrow * QLD + qcol] = qnb;
      if (t + 1 >= T1) break;
      // odd term t+1: compute from (tb, pb, buffer 1); prefetch t+2 into (ta, pa, buffer 0)
      const int t2 = t + 2 < T1 ? t + 2 : T1 - 1;
      qn = ld(cls_Q<CLS>(p, t2) + tid);
      if constexpr (DUAL) qnb = ld(cls_Q<CB_>(p, t2) + tid);
      term_setup<CLS, MO>(p, o0, t2, lo, hi, no, ta);
      if constexpr (DUAL) term_setup<CB_, MO>(p, o0, t2, lob, hib, no, wa);
      term_loadP<CLS, MO>(ta, lk, lc, pa);
      lds_barrier();
      __builtin_amdgcn_sched_barrier(0);
      term_compute<CLS, MO>(tb, pb, qbuf + 16 * QLD, lr, lk, k1, k2, k3);
      if constexpr (DUAL) term_compute<CB_, MO>(wb, pb, qb + 16 * QLD, lr, lk, b1, b2, b3);
      qbuf[qrow * QLD + qcol] = qn;
      if constexpr (DUAL) qb[qrow * QLD + qcol] = qnb;
    }
  }
  const int64_t E = bsz(p);
#pragma unroll
  for (int u = 0; u < MO; ++u) {
    if (u >= no || hi[u] <= ch * SC || lo[u] >= (ch + 1) * SC) continue;  // no term: not written
    kbe_c128 *out = base + ((int64_t)ch * nout + o0 + u) * E;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
      st(out + (4 * ti + lk) * 16 + lc, cd{k1[u][ti] - k3[u][ti], k1[u][ti] + k2[u][ti]});
  }
  if constexpr (DUAL) {
#pragma unroll
    for (int u = 0; u < MO; ++u) {
      if (u >= no || hib[u] <= lob[u] || hib[u] <= ch * SC || lob[u] >= (ch + 1) * SC) continue;
      kbe_c128 *out = baseB + ((int64_t)ch * nout + o0 + u) * E;
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
        st(out + (4 * ti + lk) * 16 + lc, cd{b1[u][ti] - b3[u][ti], b1[u][ti] + b2[u][ti]});
    }
  }
}

// One persistent launch covers every class of a call.  A task is (class k, chunk ch, output
// group block gb) with local index lb = gb * nchunk + ch; class k owns task indices
// [first[k], first[k+1]) (a multiple of 8 apart).  Task i belongs to queue i % 8; workgroup b
// serves queue b % 8 first (its XCD under round-robin placement, so the tasks of a chunk share
// one L2) and then steals from the other queues.  Queue heads live in the workspace and are
// zeroed by a fill kernel before each launch.
struct FusedPlan {
  int ncls, SC, MO;
  int cls[12], nout[12], nchunk[12], ngroup[12];
  // pair[k] >= 0: class k's tasks also compute class pair[k] (on the MFMA path C_GRU beside C_IL
  // or C_ILX, B_GRU beside B_L: the same streamed blocks and outputs), whose entry holds its
  // partial array and has no tasks of its own
  int pair[12];
  int64_t first[13];
  int64_t off[12];  // byte offset of each class's partials [nchunk][nout][N*N] in the workspace
  int64_t qoff;     // byte offset of the 8 queue heads
  int64_t sgoff;    // greater form with I^<: byte offset of the Sigma^> row (-1: none)
};

// Kernel variants ("kind"): 16 = FP64 MFMA (N = 16), 1..8 = small-block task for that N,
// 0 = generic vector-ALU task (any N).
constexpr int KIND_GENERIC = 0, KIND_MFMA = 16;

template <int KIND>
__host__ __device__ constexpr int kind_lds() {  // complex numbers of LDS per workgroup
  if constexpr (KIND == KIND_MFMA) return 4 * 16 * QLD;  // two classes' Q, double-buffered
  else if constexpr (KIND >= 1 && KIND <= 8) return SmallCfg<KIND>::LDS;
  else return 1;
}

template <int KIND, int CLS>
__device__ __forceinline__ void run_task(const Params &p, const FusedPlan &pl, int k, int64_t lb,
                                         char *ws, int lane, int wave, cd *qbuf, int *rng) {
  const int nch = pl.nchunk[k];
  const int ch = (int)(lb % nch);
  const int gb = (int)(lb / nch);
  kbe_c128 *base = (kbe_c128 *)(ws + pl.off[k]);
  if constexpr (KIND == KIND_MFMA) {
    if constexpr (CLS == C_IL || CLS == C_ILX || CLS == B_L) {
      if (pl.pair[k] >= 0) {  // C_GRU (B_GRU) on the same tasks
        constexpr int CB = CLS == B_L ? B_GRU : C_GRU;
        wg_task_mfma16<CLS, CB>(p, pl.nout[k], pl.ngroup[k], ch, gb, pl.SC, base, qbuf, rng,
                                (kbe_c128 *)(ws + pl.off[pl.pair[k]]));
        return;
      }
    }
    wg_task_mfma16<CLS>(p, pl.nout[k], pl.ngroup[k], ch, gb, pl.SC, base, qbuf, rng);
  } else if constexpr (KIND >= 1 && KIND <= 8) {
    wg_task_small<KIND, CLS>(p, pl.nout[k], pl.ngroup[k], ch, gb, pl.SC, base, qbuf, rng);
  } else {
    const int g = gb * 4 + wave;
    if (g >= pl.ngroup[k]) return;
    const int t0 = ch * pl.SC, t1 = t0 + pl.SC;
    const int o = g;
    int lo, hi;
    cls_range<CLS>(p, o, lo, hi);
    const int a = t0 > lo ? t0 : lo, b = t1 < hi ? t1 : hi;
    if (a >= b) return;
    task_generic<CLS>(p, o, a, b, base + ((int64_t)ch * pl.nout[k] + o) * bsz(p), lane);
  }
}

// ADJ selects the adjoint classes (B_*, G_MAT*) instead of the forward ones, so the two calls
// run separate, smaller kernels.
template <int KIND, bool ADJ>
__global__ void __launch_bounds__(256) stream_fused(Params p, FusedPlan pl, char *ws) {
  __shared__ cd qbuf[kind_lds<KIND>()];
  __shared__ int rng[8];
  __shared__ long long s_task;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned int *heads = (unsigned int *)(ws + pl.qoff);
  const int64_t ntask = pl.first[pl.ncls];
  const int64_t per_q = (ntask + 7) / 8;
  const int home = blockIdx.x & 7;
  for (int qi = 0; qi < 8; ++qi) {
    const int q = (home + qi) & 7;
    for (;;) {
      if (threadIdx.x == 0) {
        const unsigned int j = atomicAdd(heads + q, 1u);
        s_task = j < per_q ? (long long)j * 8 + q : -1;
      }
      lds_barrier();
      const int64_t task = s_task;
      lds_barrier();
      if (task < 0 || task >= ntask) break;  // uniform over the workgroup
      int k = 0;
      while (task >= pl.first[k + 1]) ++k;
      const int64_t lb = task - pl.first[k];
#define KBE_CASE(C) \
  case C: run_task<KIND, C>(p, pl, k, lb, ws, lane, wave, qbuf, rng); break;
      if (!ADJ) {
        switch (pl.cls[k]) {
          KBE_CASE(C_IRC) KBE_CASE(C_IRR) KBE_CASE(C_IL) KBE_CASE(C_ITV) KBE_CASE(C_JR)
          KBE_CASE(C_JM1) KBE_CASE(C_JM2)
        }
        switch (pl.cls[k]) { KBE_CASE(C_GRL) KBE_CASE(C_GRD) KBE_CASE(C_GRU) KBE_CASE(C_ILX) }
      } else {
        switch (pl.cls[k]) {
          KBE_CASE(B_R1) KBE_CASE(B_R2) KBE_CASE(B_R3) KBE_CASE(B_L) KBE_CASE(B_T1)
          KBE_CASE(B_T2A) KBE_CASE(B_T2B) KBE_CASE(G_MAT1) KBE_CASE(G_MAT2)
        }
        switch (pl.cls[k]) { KBE_CASE(B_GRL) KBE_CASE(B_GRD) KBE_CASE(B_GRU) }
        if constexpr (KIND != KIND_MFMA) {  // never planned on the MFMA path
          switch (pl.cls[k]) { KBE_CASE(B_LGU) }
        }
      }
#undef KBE_CASE
      lds_barrier();  // LDS tiles and range scratch are reused by the next task
    }
  }
}

__global__ void zero_heads(unsigned int *heads) {
  if (threadIdx.x < 8) heads[threadIdx.x] = 0u;
}

// out[x] = a[x] + b[x] over count complex numbers (the Sigma^> row of the greater form).
__global__ void __launch_bounds__(256) add_rows(const kbe_c128 *a, const kbe_c128 *b,
                                                kbe_c128 *out, int64_t count) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < count) st(out + x, ld(a + x) + ld(b + x));
}

// Chunk reduction, all outputs of a call in one launch.  Job j writes out_j[x] (=|+=) the sum,
// in increasing chunk order, of the chunks of up to three classes' partial arrays that
// intersect output o's term range; the jobs' elements are laid end to end over the grid.
constexpr int RED_PARTS = 8;  // classes summed into one output array, at most
struct RedJob {
  const kbe_c128 *a[RED_PARTS];
  int cls[RED_PARTS], nchunk[RED_PARTS];
  int nparts, nout, accumulate;
  kbe_c128 *out;
  int64_t start;  // first grid element of this job
};
constexpr int RED_JOBS = 6;  // output arrays per call, at most
struct RedAll {
  RedJob j[RED_JOBS];
  int njob, SC;
  int64_t total;
};
__global__ void __launch_bounds__(256) reduce_kernel(Params p, RedAll r) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= r.total) return;
  int jb = 0;
  while (jb + 1 < r.njob && g >= r.j[jb + 1].start) ++jb;
  const RedJob &in = r.j[jb];
  const int64_t E = bsz(p);
  const int64_t nel = (int64_t)in.nout * E;
  const int64_t x = g - in.start;
  const int o = (int)(x / E);
  cd s = czero();
  for (int k = 0; k < in.nparts; ++k) {
    int lo, hi;
    range_rt(in.cls[k], p, o, lo, hi);
    if (hi <= lo) continue;
    const int c0 = lo / r.SC;
    int c1 = (hi - 1) / r.SC;
    if (c1 > in.nchunk[k] - 1) c1 = in.nchunk[k] - 1;
    for (int c = c0; c <= c1; ++c) s = s + ld(in.a[k] + (int64_t)c * nel + x);
  }
  if (in.accumulate) s = s + ld(in.out + x);
  st(in.out + x, s);
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

// The greater form of Eq. KBE2 reads G^R in I^R (through G^> = G^< + D) and Sigma^R in I^<
// (through Sigma^> = Sigma^R + Sigma^<), which adds to the lower triangle of kp and to rdiag:
//   kp[a][b], a > b:  w[a][b] gIL(a)^dag Sigma^R(b)     (a in range; I^<)
//                    + w[n][a] Sigma^R(a)^dag gIR(b)     (b in range; D = G^R(s,m), s > m)
//                    - w[n][b] gIR(a)^dag Sigma^R(b)     (a in range; D = -G^R(m,s)^dag, s < m)
//   rdiag[a]       :  w[a][a] gIL(a)^dag Sigma^R(a)     (a in range; I^<)
//                    + w[n][a] Sigma^R(a)^dag gIR(a)     (a in range; D = G^R(m,m))
// These run after grad_generic has written the lesser-form terms of the same blocks; a block
// that pass left unwritten (no lesser-form term, overwrite mode) is written here instead.
// Blocks 0 .. (n+1)^2 - 1 are kp (a, b), then rdiag[a].
__global__ void __launch_bounds__(256) grad_greater(Params p, int64_t nblk) {
  const int E = p.N * p.N;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t blk = gid / E;
  if (blk >= nblk) return;
  const int e = (int)(gid % E), i = e / p.N, j = e % p.N;
  int kind, a, b;
  grad_block_index(p, blk, kind, a, b);
  if (kind == 0 && a <= b) return;  // the upper triangle holds G^<: no new term
  const int64_t En = bsz(p), wn = (int64_t)p.n * p.nt;
  const bool ina = a >= p.m0 && a < p.m1, inb = b >= p.m0 && b < p.m1;
  GT t[3];
  int nt = 0;
  if (p.fIL && ina) t[nt++] = GT{{p.w[(int64_t)a * p.nt + b], 0.0}, p.gIL + (a - p.m0) * En, p.ret + b * En};
  if (kind == 0) {
    if (p.fIR && inb) t[nt++] = GT{{p.w[wn + a], 0.0}, p.ret + a * En, p.gIR + (b - p.m0) * En};
    if (p.fIR && ina) t[nt++] = GT{{-p.w[wn + b], 0.0}, p.gIR + (a - p.m0) * En, p.ret + b * En};
  } else if (p.fIR && ina) {
    t[nt++] = GT{{p.w[wn + a], 0.0}, p.ret + a * En, p.gIR + (a - p.m0) * En};
  }
  if (nt == 0) return;
  cd s = czero();
  for (int q = 0; q < nt; ++q) {
    cd x = czero();
    for (int k = 0; k < p.N; ++k) x = x + cj(ld(t[q].X + k * p.N + i)) * ld(t[q].Y + k * p.N + j);
    s = s + t[q].c * x;
  }
  GT u0, u1;
  kbe_c128 *dst;
  const int before = grad_terms(p, kind, a, b, u0, u1, dst);
  if (!p.overwrite || before > 0) s = s + ld(dst + e);
  st(dst + e, s);
}

// MFMA version (N = 16).  A workgroup owns a segment of one storage row a (the kp row a, then
// the tv row a, then rdiag[a]).  Every term of that row has the form X^dag (c Y) with X one of
// four per-row blocks -- Sigma^R(a), gIR(a), gIL(a), gItv(a) -- which are staged once in LDS;
// the scalar is folded into the streamed Y.  The terms of the segment's blocks (operands,
// scalars, destination) are resolved once into LDS records.  Each wave walks every fourth block
// of the segment with the next block's Y prefetched and multiplies on v_mfma_f64_16x16x4
// (A = X^dag, one element per lane per k-chunk read from LDS; B = Y slabs straight from the
// cache), three real products per complex one, both terms into the same accumulators.
constexpr int GSEG = 64;  // blocks per workgroup segment

struct GradTerm {
  int xid;           // which staged X (0..3); -1: no term
  cd c;
  const kbe_c128 *Y;
};

// Terms of block j of row a: j < n+1 -> kp[a][j]; j < n+1+ntau -> tv[a][j-n-1]; else rdiag[a].
__device__ __forceinline__ int grad_row_terms(const Params &p, int a, int j, GradTerm &t0,
                                              GradTerm &t1, kbe_c128 *&dst) {
  const int64_t E = bsz(p);
  const int n1 = p.n + 1;
  const bool ina = a >= p.m0 && a < p.m1;
  t0.xid = t1.xid = -1;
  t0.Y = t1.Y = p.ret;
  t0.c = t1.c = czero();
  int nt = 0;
  auto push = [&](int xid, cd c, const kbe_c128 *Y) {
    if (nt == 0) t0 = GradTerm{xid, c, Y};
    else t1 = GradTerm{xid, c, Y};
    ++nt;
  };
  if (j < n1) {
    const int b = j;
    const bool inb = b >= p.m0 && b < p.m1;
    dst = p.gkp + ((int64_t)a * p.ldt + b) * E;
    if (a <= b) {
      if (p.fIR && inb) push(0, cd{p.w[(int64_t)p.n * p.nt + a], 0.0}, p.gIR + (b - p.m0) * E);
      if (p.fIR && ina && a < b) push(1, cd{-p.w[(int64_t)p.n * p.nt + b], 0.0}, p.ret + b * E);
    } else if (p.fIL && ina) {
      push(2, cd{p.w[(int64_t)a * p.nt + b], 0.0}, p.les + b * E);
    }
  } else if (j < n1 + p.ntau) {
    const int k = j - n1;
    dst = p.gtv + ((int64_t)a * p.ntau + k) * E;
    if (p.fJTV) push(0, cd{p.w[(int64_t)p.n * p.nt + a], 0.0}, p.gJ + k * E);
    if (p.fITV && ina) push(3, cd{0.0, -p.wtau[p.J - k]}, p.stv + (p.J - k) * E);
  } else {
    dst = p.grdiag + a * E;
    if (p.fIL && ina) push(2, cd{p.w[(int64_t)a * p.nt + a], 0.0}, p.les + a * E);
  }
  return nt;
}

// The greater form's extra terms (those grad_greater adds on the generic path), at most three
// per block, for grad_mfma16<1> and grad_mfma8<1>; X ids as above (0 Sigma^R(a), 1 gIR(a),
// 2 gIL(a)):
//   kp[a][b] a > b:  w[a][b] gIL(a)^dag Sigma^R(b),  w[n][a] Sigma^R(a)^dag gIR(b),
//                    -w[n][b] gIR(a)^dag Sigma^R(b)
//   rdiag[a]      :  w[a][a] gIL(a)^dag Sigma^R(a),  w[n][a] Sigma^R(a)^dag gIR(a)
__device__ __forceinline__ int grad_row_terms_gr(const Params &p, int a, int j, GradTerm &t0,
                                                 GradTerm &t1, GradTerm &t2, kbe_c128 *&dst) {
  const int64_t E = bsz(p);
  const int n1 = p.n + 1;
  const bool ina = a >= p.m0 && a < p.m1;
  const int64_t wn = (int64_t)p.n * p.nt;
  t0.xid = t1.xid = t2.xid = -1;
  t0.Y = t1.Y = t2.Y = p.ret;
  t0.c = t1.c = t2.c = czero();
  int nt = 0;
  auto push = [&](int xid, cd c, const kbe_c128 *Y) {
    const GradTerm g{xid, c, Y};
    if (nt == 0) t0 = g;
    else if (nt == 1) t1 = g;
    else t2 = g;
    ++nt;
  };
  dst = p.gkp;
  if (j < n1) {
    const int b = j;
    const bool inb = b >= p.m0 && b < p.m1;
    dst = p.gkp + ((int64_t)a * p.ldt + b) * E;
    if (a > b) {
      if (p.fIL && ina) push(2, cd{p.w[(int64_t)a * p.nt + b], 0.0}, p.ret + b * E);
      if (p.fIR && inb) push(0, cd{p.w[wn + a], 0.0}, p.gIR + (b - p.m0) * E);
      if (p.fIR && ina) push(1, cd{-p.w[wn + b], 0.0}, p.ret + b * E);
    }
  } else if (j >= n1 + p.ntau) {
    dst = p.grdiag + a * E;
    if (p.fIL && ina) push(2, cd{p.w[(int64_t)a * p.nt + a], 0.0}, p.ret + a * E);
    if (p.fIR && ina) push(0, cd{p.w[wn + a], 0.0}, p.gIR + (a - p.m0) * E);
  }
  return nt;
}

// Term sets of the gradient kernels (grad_mfma16<TS>, grad_mfma8<TS>): 0 the terms both forms
// share (at most two per block, X ids 0..3), 1 the greater form's extra terms (at most three,
// X ids 0..2), 2 both sets in one pass: the shared terms with the first parameter set's
// cotangents and the extra terms with the second's, whose gIR(a), gIL(a) are staged as X ids
// 4, 5.  At most four then: a kp block below the diagonal has one shared term and at most three
// extra ones, rdiag one and two, the other blocks no extra term.
template <int TS> struct GradSet {
  static constexpr int NT = TS == 0 ? 2 : TS == 1 ? 3 : 4;  // terms per block, at most
  static constexpr int NX = TS == 2 ? 6 : 4;                // staged X blocks per row
};

// Per-block term record of a segment, built once per workgroup in LDS.
template <int NT> struct GradRec {
  const kbe_c128 *y[NT];  // Y of each term (term 0's Y again for absent terms)
  kbe_c128 *dst;
  double cr[NT], ci[NT];  // scalars (0 for absent terms)
  int x[NT], nt;
  int acc;  // add the block's current value (accumulate mode, or a block an earlier pass wrote)
};


__device__ __forceinline__ const kbe_c128 *uniform_ptr(const kbe_c128 *q) {
  const uint64_t v = (uint64_t)q;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const kbe_c128 *)(((uint64_t)hi << 32) | lo);
}

typedef double __attribute__((ext_vector_type(4))) d4g;
__device__ __forceinline__ d4g mfma16f(double a, double b, d4g c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The record of block j0 + tid of row a.  TS = 1 adds to what the TS = 0 pass wrote
// (accumulate mode, or a block that pass reached); TS = 2 writes each block once with both
// sets' terms, the shared terms first.
template <int TS>
__device__ __forceinline__ void fill_grad_rec(const Params &p, const Params &pg, int a, int j0,
                                              int len, int tid, GradRec<GradSet<TS>::NT> &g) {
  constexpr int NT = GradSet<TS>::NT;
  GradTerm t[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) t[k] = GradTerm{-1, czero(), p.ret};
  kbe_c128 *d = p.gkp;
  int nt = 0, acc = !p.overwrite;
  if (tid < len) {
    const int j = j0 + tid;
    if constexpr (TS == 0) {
      nt = grad_row_terms(p, a, j, t[0], t[1], d);
    } else if constexpr (TS == 1) {
      nt = grad_row_terms_gr(p, a, j, t[0], t[1], t[2], d);
      GradTerm u0, u1;
      kbe_c128 *dd;
      acc = acc || grad_row_terms(p, a, j, u0, u1, dd) > 0;
    } else {
      kbe_c128 *dg = pg.gkp;
      const int n0 = grad_row_terms(p, a, j, t[0], t[1], d);
      GradTerm u[3];
      const int n1 = grad_row_terms_gr(pg, a, j, u[0], u[1], u[2], dg);
      if (n0 == 0) d = dg;  // the same block: both sets address it alike
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k >= n1) break;
        GradTerm v = u[k];
        if (v.xid > 0) v.xid += 3;  // pg's gIR(a), gIL(a)
        if (n0 == 0) t[k] = v;
        else if (n0 == 1) t[k + 1] = v;
        else t[k + 2] = v;
      }
      nt = n0 + n1;
    }
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    g.y[k] = k < nt ? t[k].Y : t[0].Y;
    g.cr[k] = k < nt ? t[k].c.re : 0.0;
    g.ci[k] = k < nt ? t[k].c.im : 0.0;
    g.x[k] = k < nt && t[k].xid >= 0 ? t[k].xid : 0;
  }
  g.dst = d;
  g.nt = nt;
  g.acc = acc;
}

// TS: the term set (GradSet); TS = 1 runs after TS = 0 and adds to what it wrote.  pg is read by
// TS = 2 only (the greater form's extra terms; its Sigma row, gradients, row range and mode are
// those of p).  The Y of terms 0 and 1 are loaded a block ahead (TS = 1: terms 0..2); TS = 2
// loads terms 2 and 3 (blocks below the diagonal and rdiag) at the start of their block, ahead
// of the next block's loads, and multiplies them after terms 0 and 1.
// ACC (TS = 0): accumulate mode; a block's current values are loaded as soon as its result is
// held, ahead of its stores (for TS = 1 and 2 the registers this needs cost more than the early
// loads gain: they load them at the store).
template <int TS, bool ACC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
grad_mfma16(Params p, Params pg, int row_len, int nseg) {
  constexpr int NTR = GradSet<TS>::NT, NX = GradSet<TS>::NX;
  constexpr int NTM = TS == 1 ? 3 : 2;  // terms whose Y are loaded a block ahead
  __shared__ cd xs[NX][16 * QLD];
  __shared__ GradRec<NTR> rec[GSEG];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lk = lane >> 4, lc = lane & 15;
  // Workgroups are dealt round-robin to the 8 XCDs; XCD x walks the segment-major range
  // [x per_xcd, (x+1) per_xcd) of (segment, row) pairs, so the column operands (Y) its L2 holds
  // belong to about one segment at a time.  The results bypass the caches (streaming stores) so
  // that they do not evict those operands.
  const int per_xcd = (int)((gridDim.x + 7) / 8);
  const int L = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (L >= (p.n + 1) * nseg) return;  // whole workgroup: before any barrier
  const int seg = L / (p.n + 1), a = L % (p.n + 1);
  const int64_t E = bsz(p);
  const bool ina = a >= p.m0 && a < p.m1;
  {  // stage the row's X blocks: Sigma^R(a), gIR(a), gIL(a), gItv(a) (zeros when absent), and
     // for TS = 2 pg's gIR(a), gIL(a)
    const int r = tid >> 4, c = tid & 15;
    xs[0][r * QLD + c] = ld(p.ret + a * E + tid);
    xs[1][r * QLD + c] = (p.fIR && ina) ? ld(p.gIR + (a - p.m0) * E + tid) : czero();
    xs[2][r * QLD + c] = (p.fIL && ina) ? ld(p.gIL + (a - p.m0) * E + tid) : czero();
    xs[3][r * QLD + c] = (p.fITV && ina) ? ld(p.gItv + (a - p.m0) * E + tid) : czero();
    if constexpr (NX > 4) {
      xs[4][r * QLD + c] = (pg.fIR && ina) ? ld(pg.gIR + (a - p.m0) * E + tid) : czero();
      xs[5][r * QLD + c] = (pg.fIL && ina) ? ld(pg.gIL + (a - p.m0) * E + tid) : czero();
    }
  }
  const int j0 = seg * GSEG, len = (j0 + GSEG < row_len ? j0 + GSEG : row_len) - j0;
  if (tid < GSEG) fill_grad_rec<TS>(p, pg, a, j0, len, tid, rec[tid]);
  __syncthreads();
  cd yn[NTM][4];  // raw Y slabs of the block after the current one
  // Every record's Y pointers are valid (a block without terms points at Sigma^R(0)), so the
  // prefetch is unconditional; past the end of the segment it re-reads the last record.
  auto fetch = [&](int q) {
    const kbe_c128 *Y[NTM];
#pragma unroll
    for (int tm = 0; tm < NTM; ++tm) Y[tm] = uniform_ptr(rec[q].y[tm]);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
#pragma unroll
      for (int tm = 0; tm < NTM; ++tm) yn[tm][kc] = ldg(Y[tm] + (4 * kc + lk) * 16 + lc);
  };
  // A block's result is held for one iteration and written one 16 x 4 slab per inner step of
  // the next block, so each wave's stores spread over its products instead of a burst.
  cd prev[4], dprev[4];
  kbe_c128 *pdst = nullptr;
  int pacc = 0;
  auto put = [&](int r) {  // rows l/16 + 4 r of the held result
    kbe_c128 *d = pdst + (lk + 4 * r) * 16 + lc;
    cd v = prev[r];
    if constexpr (ACC && TS == 0) {
      v = v + dprev[r];
    } else if (pacc) {
      v = v + ldg(d);
    }
    dvec2 w;
    w.x = v.re;
    w.y = v.im;
    __builtin_nontemporal_store(w, (g_dvec2 *)(void *)d);
  };
  // Three real products per complex one (Gauss): with A = conj(X), for each k-chunk
  //   K1 += (xr - xi) yr,   K2 += xr (yi - yr),   K3 += xi (yr + yi);
  // then Re = K1 + K3 and Im = K1 + K2.  All terms of the block share the accumulators.
  // v_mfma_f64_16x16x4: lane l supplies A[l%16][4 kc + l/16] = conj(X[4 kc + l/16][l%16]) and
  // B[4 kc + l/16][l%16] = c Y[..], and holds D[l/16 + 4 r][l%16].
  d4g k1, k2, k3;
  auto product = [&](const cd *x, cd yv, int kc) {
    const cd u = x[(4 * kc + lk) * QLD + lc];
    const double ys = yv.im - yv.re, yp = yv.re + yv.im;
    __builtin_amdgcn_sched_barrier(0);
    k1 = mfma16f(u.re - u.im, yv.re, k1);
    k2 = mfma16f(u.re, ys, k2);
    k3 = mfma16f(u.im, yp, k3);
    __builtin_amdgcn_sched_barrier(0);
  };
  int q = __builtin_amdgcn_readfirstlane(wave);
  if (q < len) fetch(q);
  for (; q < len; q += 4) {
    const int cnt = __builtin_amdgcn_readfirstlane(rec[q].nt);
    kbe_c128 *const cdst = (kbe_c128 *)uniform_ptr(rec[q].dst);
    cd cs[NTR];
    const cd *xt[NTR];
#pragma unroll
    for (int tm = 0; tm < NTR; ++tm) {
      cs[tm] = cd{rec[q].cr[tm], rec[q].ci[tm]};
      xt[tm] = xs[__builtin_amdgcn_readfirstlane(rec[q].x[tm])];
    }
    cd y[NTM][4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
#pragma unroll
      for (int tm = 0; tm < NTM; ++tm) y[tm][kc] = cs[tm] * yn[tm][kc];
    cd z[2][4];  // TS = 2: raw Y of terms 2 and 3 of this block
    if constexpr (TS == 2) {
      if (cnt > 2) {  // wave-uniform; term 3's Y is term 0's when absent
        const kbe_c128 *Z0 = uniform_ptr(rec[q].y[2]), *Z1 = uniform_ptr(rec[q].y[3]);
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          z[0][kc] = ldg(Z0 + (4 * kc + lk) * 16 + lc);
          z[1][kc] = ldg(Z1 + (4 * kc + lk) * 16 + lc);
        }
      }
    }
    // issue the next block's loads before this block's products and stores
    fetch(q + 4 < len ? q + 4 : len - 1);
    if (cnt == 0) continue;
    k1 = d4g{0, 0, 0, 0};
    k2 = d4g{0, 0, 0, 0};
    k3 = d4g{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
#pragma unroll
      for (int term = 0; term < NTM; ++term) {
        if (term >= cnt) break;  // wave-uniform
        product(xt[term], y[term][kc], kc);
      }
      if (pdst) put(kc);
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (TS == 2) {
      if (cnt > 2) {
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
#pragma unroll
          for (int t2 = 0; t2 < 2; ++t2) {
            if (2 + t2 >= cnt) break;  // wave-uniform
            product(xt[2 + t2], cs[2 + t2] * z[t2][kc], kc);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) prev[r] = cd{k1[r] + k3[r], k1[r] + k2[r]};
    pdst = cdst;
    if constexpr (ACC && TS == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) dprev[r] = ldg(pdst + (lk + 4 * r) * 16 + lc);
    } else if constexpr (TS == 1) {
      pacc = __builtin_amdgcn_readfirstlane(rec[q].acc);
    } else if constexpr (TS == 2) {
      pacc = !p.overwrite;
    }
  }
  if (pdst) {
#pragma unroll
    for (int r = 0; r < 4; ++r) put(r);
  }
}

// MFMA version for 5 <= N <= 8.  Blocks are zero-padded to 8 x 8 and one v_mfma_f64_4x4x4
// instruction computes all four 4 x 4 tiles (ti, tj) of an 8 x 8 product (instruction block
// b = 2 ti + tj), so a block costs two k-chunks of three real products per term.  Lane roles:
//   A[b][i][k] = conj(X[4 kc + k][4 ti + i])  at lane 4b + i + 16k   (read from LDS),
//   B[b][k][j] = c Y[4 kc + k][4 tj + j]      at lane 4b + j + 16k   (loaded from the cache),
//   D[b][i][j] = out[4 ti + i][4 tj + j]      at lane 4b + j + 16i,
// so lanes 8r .. 8r+7 of a store hold a whole row of the block (128 contiguous bytes at N = 8).
// Work split, records, prefetch and streaming stores as in grad_mfma16.
constexpr int GSEG8 = 64;   // blocks per workgroup segment (64 beat 32, 128 and 256)
constexpr int XLD8 = 9;     // LDS row stride of a staged 8x8 block, in complex numbers

// TS: the term set (GradSet).  pg is read by TS = 2 only (the greater form's extra terms; its Sigma
// row, gradients, row range and mode are those of p).  ACC: blocks add to their current values
// (accumulate mode; TS = 1: the blocks whose record says so), which are loaded with the block's
// operands.  Each wave walks every fourth block of the segment with the next block's loads in
// flight, alternating between two register sets (the loop is unrolled by two, so no prefetched
// value is copied: a copy would wait for its load); every load is unconditional (an absent
// term re-reads term 0's block, which the cache holds), so each wait covers exactly one set.
template <int TS, bool ACC>
__global__ void __launch_bounds__(256) grad_mfma8(Params p, Params pg, int row_len, int nseg) {
  constexpr int NTM = GradSet<TS>::NT, NX = GradSet<TS>::NX;
  __shared__ cd xs[NX][8 * XLD8];
  __shared__ GradRec<NTM> rec[GSEG8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = p.N;
  const int per_xcd = (int)((gridDim.x + 7) / 8);
  const int L = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (L >= (p.n + 1) * nseg) return;  // whole workgroup: before any barrier
  const int seg = L / (p.n + 1), a = L % (p.n + 1);
  const int64_t E = bsz(p);
  const bool ina = a >= p.m0 && a < p.m1;
  // stage the row's X blocks (Sigma^R(a), gIR(a), gIL(a), gItv(a); TS = 2 also pg's gIR(a),
  // gIL(a)), zero-padded to 8 x 8
  for (int s = tid; s < NX * 64; s += 256) {
    const int x = s >> 6, r = (s >> 3) & 7, c = s & 7;
    const bool present = x == 0 || (x == 1 && p.fIR && ina) || (x == 2 && p.fIL && ina) ||
                         (x == 3 && p.fITV && ina) || (x == 4 && pg.fIR && ina) ||
                         (x == 5 && pg.fIL && ina);
    const kbe_c128 *X = x == 0 ? p.ret + a * E
                        : x == 1 ? p.gIR + (a - p.m0) * E
                        : x == 2 ? p.gIL + (a - p.m0) * E
                        : x == 3 ? p.gItv + (a - p.m0) * E
                        : x == 4 ? pg.gIR + (a - p.m0) * E
                                 : pg.gIL + (a - p.m0) * E;
    xs[x][r * XLD8 + c] = (present && r < N && c < N) ? ld(X + r * N + c) : czero();
  }
  const int j0 = seg * GSEG8, len = (j0 + GSEG8 < row_len ? j0 + GSEG8 : row_len) - j0;
  if (tid < GSEG8) fill_grad_rec<TS>(p, pg, a, j0, len, tid, rec[tid]);
  __syncthreads();
  const int lj = lane & 3, lb = (lane >> 2) & 3, lk = lane >> 4;
  const int ti = lb >> 1, tj = lb & 1;
  // B element of k-chunk kc: row 4 kc + lk, column 4 tj + lj (zero outside N x N)
  const int bc = 4 * tj + lj;
  const bool bv0 = lk < N && bc < N, bv1 = 4 + lk < N && bc < N;
  const int bo0 = bv0 ? lk * N + bc : 0, bo1 = bv1 ? (4 + lk) * N + bc : 0;
  // D element: row 4 ti + lk, column 4 tj + lj
  const bool dv = 4 * ti + lk < N && bc < N;
  const int dof = dv ? (4 * ti + lk) * N + bc : 0;
  struct Ops {
    cd y[NTM][2];  // raw Y of [term][kc]
    cd d;          // the destination's current value (ACC)
  };
  auto fetch = [&](int q, Ops &f) {
#pragma unroll
    for (int tm = 0; tm < NTM; ++tm) {
      const kbe_c128 *Y = uniform_ptr(rec[q].y[tm]);
      f.y[tm][0] = ldg(Y + bo0);
      f.y[tm][1] = ldg(Y + bo1);
    }
    if constexpr (ACC) f.d = ldg(uniform_ptr(rec[q].dst) + dof);
  };
  // Registers that a store reads may be rewritten only after the store, and the wait for it
  // counts every earlier load too.  So the stored value is not formed in f.d's registers, and
  // each set's stored value (w) and address (wp) stay live until the other set's loads have
  // been issued.
  auto keep = [](const dvec2 &w) { asm volatile("" ::"v"(w.x), "v"(w.y)); };
  auto keep_p = [](uint64_t a) { asm volatile("" ::"v"(a)); };
  auto work = [&](int q, const Ops &f, dvec2 &w, uint64_t &wp) {
    const int cnt = __builtin_amdgcn_readfirstlane(rec[q].nt);
    if (cnt == 0) return;
    kbe_c128 *const cdst = (kbe_c128 *)uniform_ptr(rec[q].dst);
    // three real products per complex one, A = conj(X) (see grad_mfma16):
    //   K1 += (xr - xi) yr,  K2 += xr (yi - yr),  K3 += xi (yr + yi);  Re = K1 + K3, Im = K1 + K2
    double k1 = 0.0, k2 = 0.0, k3 = 0.0;
#pragma unroll
    for (int term = 0; term < NTM; ++term) {
      if (term >= cnt) break;  // wave-uniform
      const cd c{rec[q].cr[term], rec[q].ci[term]};
      const cd *x = xs[__builtin_amdgcn_readfirstlane(rec[q].x[term])];
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        const cd u = x[(4 * kc + lk) * XLD8 + 4 * ti + lj];
        const cd v = c * ((kc == 0 ? bv0 : bv1) ? f.y[term][kc] : czero());
        k1 = mfma4(u.re - u.im, v.re, k1);
        k2 = mfma4(u.re, v.im - v.re, k2);
        k3 = mfma4(u.im, v.re + v.im, k3);
      }
    }
    cd r{k1 + k3, k1 + k2};
    if constexpr (ACC) {
      if (TS != 1 || __builtin_amdgcn_readfirstlane(rec[q].acc)) r = r + f.d;
    }
    w.x = r.re;
    w.y = r.im;
    wp = (uint64_t)(cdst + dof);
    if (dv) __builtin_nontemporal_store(w, (g_dvec2 *)wp);
    if constexpr (ACC) keep(dvec2{f.d.re, f.d.im});  // the sum is not formed in f.d's registers
  };
  Ops A, B;
  dvec2 wA{0.0, 0.0}, wB{0.0, 0.0};  // each set's last stored value and its address
  uint64_t pA = 0, pB = 0;
  int q = __builtin_amdgcn_readfirstlane(wave);
  if (q < len) fetch(q, A);
  for (; q < len; q += 8) {
    // block q from A; block q + 4's loads into B first (past the segment: the last block again)
    fetch(q + 4 < len ? q + 4 : len - 1, B);
    keep(wB);
    keep_p(pB);
    __builtin_amdgcn_sched_barrier(0);
    work(q, A, wA, pA);
    __builtin_amdgcn_sched_barrier(0);
    if (q + 4 >= len) break;
    fetch(q + 8 < len ? q + 8 : len - 1, A);
    keep(wA);
    keep_p(pA);
    __builtin_amdgcn_sched_barrier(0);
    work(q + 4, B, wB, pB);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ------------------------------------------------------------------------------------------
// Host side: chunking, workspace layout and launches.
// ------------------------------------------------------------------------------------------
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static int path_kind(int N, unsigned flags) {
  if (flags & KBE_FORCE_GENERIC) return KIND_GENERIC;
  if (N == 16) return KIND_MFMA;
  return N <= 8 ? N : KIND_GENERIC;
}

static int chunk_terms(int N, int kind) {
  if (kind == KIND_MFMA) return 256;
  if (kind != KIND_GENERIC) return N >= 5 ? 128 : (N >= 3 ? 256 : 1024);
  const int E = N * N;
  return E >= 64 ? 256 : (E >= 16 ? 1024 : 4096);
}

template <int... Ns>
static int small_mo(int N, std::integer_sequence<int, Ns...>) {
  int mo = 1;
  ((mo = (N == Ns + 1 ? SmallCfg<Ns + 1>::MO : mo)), ...);
  return mo;
}

static int outputs_per_wave(int N, int kind) {
  if (kind == KIND_MFMA) return MO_MFMA;
  if (kind == KIND_GENERIC) return 1;
  return small_mo(N, std::make_integer_sequence<int, 8>{});
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
  const int64_t tasks = (int64_t)pl.nchunk[k] * ((pl.ngroup[k] + 3) / 4);
  pl.first[k + 1] = pl.first[k] + (tasks + 7) / 8 * 8;
  off += al256(sizeof(kbe_c128) * (size_t)pl.nchunk[k] * nout * E);
}

static FusedPlan plan_init(int N, int kind, int SC) {
  FusedPlan pl{};
  pl.SC = SC;
  pl.MO = outputs_per_wave(N, kind);
  for (int k = 0; k < 12; ++k) pl.pair[k] = -1;
  return pl;
}

// Class cls computed by the tasks of entry partner (same outputs and chunks): an entry for its
// partial array, with no tasks.
static void plan_add_pair(FusedPlan &pl, int cls, int partner, int E, size_t &off) {
  const int k = pl.ncls++;
  pl.cls[k] = cls;
  pl.nout[k] = pl.nout[partner];
  pl.nchunk[k] = pl.nchunk[partner];
  pl.ngroup[k] = pl.ngroup[partner];
  pl.off[k] = (int64_t)off;
  pl.first[k + 1] = pl.first[k];
  off += al256(sizeof(kbe_c128) * (size_t)pl.nchunk[k] * pl.nout[k] * E);
  pl.pair[partner] = k;
}

// Small-block calls with few tasks (the early rows of a propagation) use shorter term chunks, so
// that the work spreads over more workgroups and no single task sets the length of the call: the
// chunk is halved, down to 32 terms, while the plan has fewer than MIN_TASKS tasks.  The choice
// depends only on the call's shape, so the workspace query and the launch agree.
constexpr int64_t MIN_TASKS = 1024;
template <typename F>
static size_t plan_sized(int N, int kind, FusedPlan &pl, F build) {
  int sc = chunk_terms(N, kind);
  size_t off = build(sc);
  if (kind >= 1 && kind <= 8)
    while (sc > 32 && pl.first[pl.ncls] < MIN_TASKS) {
      sc /= 2;
      off = build(sc);
    }
  return off;
}

static size_t plan_forward_sc(int N, int ntau, int n, int m0, int m1, unsigned flags, int kind,
                              int SC, FusedPlan &pl) {
  pl = plan_init(N, kind, SC);
  const int E = N * N, M = m1 - m0;
  size_t off = 0;
  const bool th = ntau > 0;
  const bool both = flags & KBE_INT_BOTH;
  const bool gr = (flags & KBE_GREATER) || both;
  // MFMA path: C_GRU rides on the tasks of the greater form's I^< class (C_IL on the Sigma^> row,
  // or C_ILX beside the lesser form), which stream the same blocks kp[m][s], s < m
  const bool pairgu = gr && kind == KIND_MFMA && (flags & KBE_OUT_IR) && (flags & KBE_OUT_IL) &&
                      m1 > 1 && M > 0;
  if (flags & KBE_OUT_IR) {
    plan_add(pl, C_IRC, M, m1, E, off);
    if (n > m0) plan_add(pl, C_IRR, M, n + 1, E, off);
    if (gr) {
      if (n > m0) plan_add(pl, C_GRL, M, n + 1, E, off);
      plan_add(pl, C_GRD, M, m1, E, off);
      if (m1 > 1 && !pairgu) plan_add(pl, C_GRU, M, m1 - 1, E, off);
    }
  }
  if (flags & KBE_OUT_IL) plan_add(pl, C_IL, M, m1, E, off);  // greater form: Q = Sigma^> row
  if (both && (flags & KBE_OUT_IL)) plan_add(pl, C_ILX, M, m1, E, off);
  if (pairgu) plan_add_pair(pl, C_GRU, pl.ncls - 1, E, off);
  if ((flags & KBE_OUT_ITV) && th) plan_add(pl, C_ITV, M, ntau, E, off);
  if ((flags & KBE_OUT_JTV) && th) {
    plan_add(pl, C_JR, ntau, n + 1, E, off);
    plan_add(pl, C_JM1, ntau, ntau, E, off);
    plan_add(pl, C_JM2, ntau, ntau, E, off);
  }
  pl.qoff = (int64_t)off;
  off += 256;
  pl.sgoff = -1;
  if (gr && (flags & KBE_OUT_IL) && m1 > 0) {  // Sigma^> = Sigma^R + Sigma^< at t_s, s < m1
    pl.sgoff = (int64_t)off;
    off += al256(sizeof(kbe_c128) * (size_t)m1 * E);
  }
  return off;
}

static size_t plan_forward(int N, int ntau, int n, int m0, int m1, unsigned flags, int kind,
                           FusedPlan &pl) {
  return plan_sized(N, kind, pl, [&](int sc) {
    return plan_forward_sc(N, ntau, n, m0, m1, flags, kind, sc, pl);
  });
}

static size_t plan_adjoint_sc(int N, int ntau, int n, int m0, int m1, unsigned flags, int kind,
                              int SC, FusedPlan &pl) {
  pl = plan_init(N, kind, SC);
  const int E = N * N;
  size_t off = 0;
  const bool th = ntau > 0, M = m1 > m0;
  const bool fITV = (flags & KBE_OUT_ITV) && th, fJTV = (flags & KBE_OUT_JTV) && th;
  // B_L and B_GRU stream the same blocks kp[m][s], m > s, into the same output s: on the MFMA
  // path B_GRU rides on B_L's tasks (FusedPlan::pair)
  const bool pairgu = (flags & KBE_GREATER) && kind == KIND_MFMA && (flags & KBE_OUT_IR) &&
                      (flags & KBE_OUT_IL) && M;
  if (flags & KBE_INT_GREXTRA) {  // only the greater form's terms beyond the lesser form's
    // one class for B_L and B_GRU when they share their operand (small-block and generic tasks)
    const bool merge = (flags & KBE_INT_SAMECOT) && kind != KIND_MFMA &&
                       (flags & KBE_OUT_IR) && (flags & KBE_OUT_IL);
    if ((flags & KBE_OUT_IR) && M) {
      plan_add(pl, B_GRL, n + 1, m1, E, off);
      plan_add(pl, B_GRD, n + 1, m1, E, off);
      if (!merge && !pairgu) plan_add(pl, B_GRU, n + 1, m1, E, off);
    }
    if ((flags & KBE_OUT_IL) && M) plan_add(pl, merge ? B_LGU : B_L, n + 1, m1, E, off);
    if (pairgu) plan_add_pair(pl, B_GRU, pl.ncls - 1, E, off);
    pl.qoff = (int64_t)off;
    return off + 256;
  }
  if ((flags & KBE_OUT_IR) && M) {
    plan_add(pl, B_R1, n + 1, m1, E, off);
    plan_add(pl, B_R2, n + 1, m1, E, off);
    if (flags & KBE_GREATER) {
      plan_add(pl, B_GRL, n + 1, m1, E, off);
      plan_add(pl, B_GRD, n + 1, m1, E, off);
      if (!pairgu) plan_add(pl, B_GRU, n + 1, m1, E, off);
    }
  }
  if (fJTV) plan_add(pl, B_R3, n + 1, ntau, E, off);
  if ((flags & KBE_OUT_IL) && M) plan_add(pl, B_L, n + 1, m1, E, off);
  if (pairgu) plan_add_pair(pl, B_GRU, pl.ncls - 1, E, off);
  if (fITV && M) plan_add(pl, B_T1, ntau, m1, E, off);
  if (fJTV) {
    plan_add(pl, B_T2A, ntau, ntau, E, off);
    plan_add(pl, B_T2B, ntau, ntau, E, off);
    plan_add(pl, G_MAT1, ntau, ntau, E, off);
    plan_add(pl, G_MAT2, ntau, ntau, E, off);
  }
  pl.qoff = (int64_t)off;
  return off + 256;
}

static size_t plan_adjoint(int N, int ntau, int n, int m0, int m1, unsigned flags, int kind,
                           FusedPlan &pl) {
  return plan_sized(N, kind, pl, [&](int sc) {
    return plan_adjoint_sc(N, ntau, n, m0, m1, flags, kind, sc, pl);
  });
}

size_t collision_ws_bytes(int N, int nt, int ntau, int n, int m0, int m1, unsigned flags) {
  (void)nt;
  FusedPlan pl;
  return plan_forward(N, ntau, n, m0, m1, flags, path_kind(N, flags), pl);
}

size_t collision_vjp_ws_bytes(int N, int nt, int ntau, int n, int m0, int m1, unsigned flags) {
  (void)nt;
  FusedPlan pl;
  const size_t b = plan_adjoint(N, ntau, n, m0, m1, flags, path_kind(N, flags), pl);
  if (!(flags & KBE_INT_GREXTRA)) return b;
  // the launch merges two classes when the cotangents are one array (fewer tasks, possibly
  // shorter chunks): enough for either plan
  const size_t b2 = plan_adjoint(N, ntau, n, m0, m1, flags | KBE_INT_SAMECOT, path_kind(N, flags), pl);
  return b > b2 ? b : b2;
}

// The most any whole-row call (m in [0, n]) at n < nt needs: what a propagation over nt points
// reserves for its collision calls.
// (one plan per row; memoised per shape, since the propagations query it at every call)
static size_t ws_rows(int N, int nt, int ntau, unsigned flags, bool adjoint) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, unsigned, bool>, size_t> memo;
  const auto key = std::make_tuple(N, nt, ntau, flags, adjoint);
  {
    std::lock_guard<std::mutex> g(mu);
    const auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  size_t b = 0;
  for (int n = 0; n < nt; ++n) {
    const size_t x = adjoint ? collision_vjp_ws_bytes(N, nt, ntau, n, 0, n + 1, flags)
                             : collision_ws_bytes(N, nt, ntau, n, 0, n + 1, flags);
    b = x > b ? x : b;
  }
  std::lock_guard<std::mutex> g(mu);
  memo[key] = b;
  return b;
}
size_t collision_ws_bytes_rows(int N, int nt, int ntau, unsigned flags) {
  return ws_rows(N, nt, ntau, flags, false);
}
size_t collision_vjp_ws_bytes_rows(int N, int nt, int ntau, unsigned flags) {
  return ws_rows(N, nt, ntau, flags, true);
}

// Resident workgroups of the persistent kernel on the current device (queried once per
// device and kernel variant).
template <int KIND, bool ADJ>
static int persistent_grid() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
  int &c = cached[dev];
  if (c == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stream_fused<KIND, ADJ>, 256, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    c = cus * per_cu;
  }
  return c;
}

template <int KIND, bool ADJ>
static void launch_fused(const Params &p, const FusedPlan &pl, char *ws, hipStream_t st) {
  const int64_t ntask = pl.first[pl.ncls];
  if (ntask == 0) return;
  hipLaunchKernelGGL(zero_heads, dim3(1), dim3(64), 0, st, (unsigned int *)(ws + pl.qoff));
  int64_t grid = persistent_grid<KIND, ADJ>();
  if (grid > ntask) grid = ntask;
  hipLaunchKernelGGL((stream_fused<KIND, ADJ>), dim3((unsigned)grid), dim3(256), 0, st, p, pl, ws);
}

template <bool ADJ>
static void launch_kind(int kind, const Params &p, const FusedPlan &pl, char *ws, hipStream_t st) {
  switch (kind) {
    case KIND_MFMA: launch_fused<KIND_MFMA, ADJ>(p, pl, ws, st); break;
    case 1: launch_fused<1, ADJ>(p, pl, ws, st); break;
    case 2: launch_fused<2, ADJ>(p, pl, ws, st); break;
    case 3: launch_fused<3, ADJ>(p, pl, ws, st); break;
    case 4: launch_fused<4, ADJ>(p, pl, ws, st); break;
    case 5: launch_fused<5, ADJ>(p, pl, ws, st); break;
    case 6: launch_fused<6, ADJ>(p, pl, ws, st); break;
    case 7: launch_fused<7, ADJ>(p, pl, ws, st); break;
    case 8: launch_fused<8, ADJ>(p, pl, ws, st); break;
    default: launch_fused<KIND_GENERIC, ADJ>(p, pl, ws, st); break;
  }
}

// Reduce the listed classes (those present in the plan) into out[nout][E].
// Queue a reduction of the listed classes (those present in the plan) into out[nout][E].
static void reduce_into(const Params &p, const FusedPlan &pl, std::initializer_list<int> classes,
                        char *ws, int nout, kbe_c128 *out, bool accumulate, RedAll &r) {
  const int64_t nel = (int64_t)nout * p.N * p.N;
  if (nel == 0 || r.njob >= RED_JOBS) return;
  RedJob &in = r.j[r.njob++];
  in = RedJob{};
  for (int c : classes)
    for (int k = 0; k < pl.ncls; ++k)
      if (pl.cls[k] == c && in.nparts < RED_PARTS) {
        in.a[in.nparts] = (const kbe_c128 *)(ws + pl.off[k]);
        in.cls[in.nparts] = c;
        in.nchunk[in.nparts] = pl.nchunk[k];
        ++in.nparts;
      }
  in.nout = nout;
  in.accumulate = accumulate ? 1 : 0;
  in.out = out;
  in.start = r.total;
  r.total += nel;
}

static void reduce_launch(const Params &p, const RedAll &r, hipStream_t st) {
  if (r.total == 0) return;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)((r.total + 255) / 256)), dim3(256), 0, st, p,
                     r);
}

hipError_t launch_collision(const Params &p, unsigned flags, kbe_c128 *IR, kbe_c128 *IL,
                            kbe_c128 *Itv, kbe_c128 *Jtv, void *ws, hipStream_t st) {
  const int kind = path_kind(p.N, flags);
  FusedPlan pl;
  plan_forward(p.N, p.ntau, p.n, p.m0, p.m1, flags, kind, pl);
  char *w = (char *)ws;
  if (pl.sgoff >= 0) {  // greater form: I^< reads Sigma^> = Sigma^R + Sigma^< through C_IL
    kbe_c128 *sg = (kbe_c128 *)(w + pl.sgoff);
    const int64_t cnt = (int64_t)p.m1 * p.N * p.N;
    hipLaunchKernelGGL(add_rows, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, p.ret,
                       p.les, sg, cnt);
    Params pg = p;
    pg.les = sg;
    launch_kind<false>(kind, pg, pl, w, st);
  } else {
    launch_kind<false>(kind, p, pl, w, st);
  }
  const int M = p.m1 - p.m0;
  RedAll r{};
  r.SC = pl.SC;
  if (flags & KBE_OUT_IR) reduce_into(p, pl, {C_IRC, C_IRR, C_GRL, C_GRD, C_GRU}, w, M, IR, false, r);
  if (flags & KBE_OUT_IL) reduce_into(p, pl, {C_IL}, w, M, IL, false, r);
  if (flags & KBE_OUT_ITV) reduce_into(p, pl, {C_ITV}, w, M, Itv, false, r);
  if ((flags & KBE_OUT_JTV) && p.ntau > 0) reduce_into(p, pl, {C_JR, C_JM1, C_JM2}, w, p.ntau, Jtv, false, r);
  reduce_launch(p, r, st);
  return hipGetLastError();
}

hipError_t launch_collision_both(const Params &p, kbe_c128 *IRl, kbe_c128 *ILl, kbe_c128 *Itv,
                                 kbe_c128 *Jtv, kbe_c128 *IRg, kbe_c128 *ILg, void *ws,
                                 hipStream_t st) {
  const unsigned flags = KBE_OUT_ALL | KBE_INT_BOTH;
  const int kind = path_kind(p.N, flags);
  FusedPlan pl;
  plan_forward(p.N, p.ntau, p.n, p.m0, p.m1, flags, kind, pl);
  char *w = (char *)ws;
  Params pg = p;
  if (pl.sgoff >= 0) {  // C_ILX reads Sigma^> = Sigma^R + Sigma^<, formed once
    kbe_c128 *sg = (kbe_c128 *)(w + pl.sgoff);
    const int64_t cnt = (int64_t)p.m1 * p.N * p.N;
    hipLaunchKernelGGL(add_rows, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, p.ret,
                       p.les, sg, cnt);
    pg.sgt = sg;
  }
  launch_kind<false>(kind, pg, pl, w, st);
  const int M = p.m1 - p.m0;
  RedAll r{};
  r.SC = pl.SC;
  reduce_into(p, pl, {C_IRC, C_IRR}, w, M, IRl, false, r);
  reduce_into(p, pl, {C_IRC, C_IRR, C_GRL, C_GRD, C_GRU}, w, M, IRg, false, r);
  reduce_into(p, pl, {C_IL}, w, M, ILl, false, r);
  reduce_into(p, pl, {C_ILX}, w, M, ILg, false, r);
  if (p.ntau > 0) {
    reduce_into(p, pl, {C_ITV}, w, M, Itv, false, r);
    reduce_into(p, pl, {C_JR, C_JM1, C_JM2}, w, p.ntau, Jtv, false, r);
  }
  reduce_launch(p, r, st);
  return hipGetLastError();
}

namespace {
// The self-energy (and G^M) gradients of an adjoint call: the stream task pass and its reduces.
void vjp_sums(const Params &p, unsigned flags, kbe_c128 *gmat, const kbe_sigma_row *gS,
              void *ws, hipStream_t st) {
  const int kind = path_kind(p.N, flags);
  FusedPlan pl;
  const unsigned pf =
      flags | (((flags & KBE_INT_GREXTRA) && p.gIR == p.gIL) ? KBE_INT_SAMECOT : 0u);
  plan_adjoint(p.N, p.ntau, p.n, p.m0, p.m1, pf, kind, pl);
  char *w = (char *)ws;
  launch_kind<true>(kind, p, pl, w, st);
  // self-energy gradients: overwritten
  RedAll r{};
  r.SC = pl.SC;
  const bool extra = flags & KBE_INT_GREXTRA;
  if (extra) {  // the Sigma^R part of Sigma^> in I^< and the G^R terms; nothing reaches Sigma^<
    reduce_into(p, pl, {B_GRL, B_GRD, B_GRU, B_L, B_LGU}, w, p.n + 1, gS->ret, false, r);
    reduce_into(p, pl, {}, w, p.n + 1, gS->les, false, r);
    reduce_launch(p, r, st);
  } else if (flags & KBE_GREATER)  // Sigma^> = Sigma^R + Sigma^< in I^<: its terms also reach gSigma^R
    reduce_into(p, pl, {B_R1, B_R2, B_R3, B_GRL, B_GRD, B_GRU, B_L}, w, p.n + 1, gS->ret, false, r);
  else
    reduce_into(p, pl, {B_R1, B_R2, B_R3}, w, p.n + 1, gS->ret, false, r);
  if (!extra) {
    reduce_into(p, pl, {B_L}, w, p.n + 1, gS->les, false, r);
    if (p.ntau > 0) reduce_into(p, pl, {B_T1, B_T2A, B_T2B}, w, p.ntau, gS->tv, false, r);
    if (p.fJTV) reduce_into(p, pl, {G_MAT1, G_MAT2}, w, p.ntau, gmat, !p.overwrite, r);
    reduce_launch(p, r, st);
  }
}

void launch_grad16(int TS, const Params &p, const Params &pg, int row_len, hipStream_t st) {
  const int nseg = (row_len + GSEG - 1) / GSEG;
  const int64_t tasks = (int64_t)(p.n + 1) * nseg;
  const dim3 grid((unsigned)(8 * ((tasks + 7) / 8)));
  if (TS == 0 && p.overwrite)
    hipLaunchKernelGGL((grad_mfma16<0, false>), grid, dim3(256), 0, st, p, pg, row_len, nseg);
  else if (TS == 0)
    hipLaunchKernelGGL((grad_mfma16<0, true>), grid, dim3(256), 0, st, p, pg, row_len, nseg);
  else if (TS == 1)
    hipLaunchKernelGGL((grad_mfma16<1, false>), grid, dim3(256), 0, st, p, pg, row_len, nseg);
  else
    hipLaunchKernelGGL((grad_mfma16<2, false>), grid, dim3(256), 0, st, p, pg, row_len, nseg);
}

void launch_grad8(int TS, const Params &p, const Params &pg, int row_len, hipStream_t st) {
  const int nseg = (row_len + GSEG8 - 1) / GSEG8;
  const int64_t tasks = (int64_t)(p.n + 1) * nseg;
  const dim3 grid((unsigned)(8 * ((tasks + 7) / 8)));
  const bool acc = !p.overwrite;
  if (TS == 0 && acc)
    hipLaunchKernelGGL((grad_mfma8<0, true>), grid, dim3(256), 0, st, p, pg, row_len, nseg);
  else if (TS == 0)
    hipLaunchKernelGGL((grad_mfma8<0, false>), grid, dim3(256), 0, st, p, pg, row_len, nseg);
  else if (TS == 1)  // the records say which blocks add
    hipLaunchKernelGGL((grad_mfma8<1, true>), grid, dim3(256), 0, st, p, pg, row_len, nseg);
  else if (acc)
    hipLaunchKernelGGL((grad_mfma8<2, true>), grid, dim3(256), 0, st, p, pg, row_len, nseg);
  else
    hipLaunchKernelGGL((grad_mfma8<2, false>), grid, dim3(256), 0, st, p, pg, row_len, nseg);
}

// The Green's-function gradients of an adjoint call.  The greater form adds its extra terms
// (those beyond the terms the forms share); at 5 <= N <= 8 both sets go in one pass.
void vjp_grads(const Params &p, unsigned flags, hipStream_t st) {
  const int kind = path_kind(p.N, flags);
  const bool extra = flags & KBE_INT_GREXTRA;
  const int64_t n1 = p.n + 1;
  const int64_t nblk = n1 * n1 + n1 + (p.ntau > 0 ? n1 * p.ntau : 0);
  const int row_len = p.n + 2 + p.ntau;  // kp row, tv row, rdiag
  if (kind == KIND_MFMA) {
    launch_grad16(extra ? 1 : (flags & KBE_GREATER) ? 2 : 0, p, p, row_len, st);
  } else if (kind >= 5 && kind <= 8) {
    launch_grad8(extra ? 1 : (flags & KBE_GREATER) ? 2 : 0, p, p, row_len, st);
  } else {
    if (!extra) {
      const int64_t th = nblk * p.N * p.N;
      hipLaunchKernelGGL(grad_generic, dim3((unsigned)((th + 255) / 256)), dim3(256), 0, st, p,
                         nblk);
    }
    if (flags & KBE_GREATER) {  // adds to what it wrote
      const int64_t nk = n1 * n1 + n1, tk = nk * p.N * p.N;  // kp and rdiag blocks
      hipLaunchKernelGGL(grad_greater, dim3((unsigned)((tk + 255) / 256)), dim3(256), 0, st, p,
                         nk);
    }
  }
}
}  // namespace

hipError_t launch_collision_vjp(const Params &p, unsigned flags, kbe_c128 *gmat,
                                const kbe_sigma_row *gS, void *ws, hipStream_t st) {
  vjp_sums(p, flags, gmat, gS, ws, st);
  vjp_grads(p, flags, st);
  return hipGetLastError();
}

hipError_t launch_collision_vjp_pair(const Params &p, unsigned flags, const Params &pg,
                                     unsigned gflags, kbe_c128 *gmat, const kbe_sigma_row *gS,
                                     const kbe_sigma_row *gSg, void *ws, hipStream_t st) {
  vjp_sums(p, flags, gmat, gS, ws, st);
  vjp_sums(pg, gflags, gmat, gSg, ws, st);  // stream-ordered after the first pass's reduces
  const int kind = path_kind(p.N, flags);
  // one pass when the two sets share everything but their cotangents and flags
  const bool same = p.N == pg.N && p.n == pg.n && p.m0 == pg.m0 && p.m1 == pg.m1 &&
                    p.ntau == pg.ntau && p.ret == pg.ret && p.w == pg.w && p.gkp == pg.gkp &&
                    p.grdiag == pg.grdiag && p.gtv == pg.gtv && p.ldt == pg.ldt &&
                    p.overwrite == pg.overwrite;
  if (same && (kind == KIND_MFMA || (kind >= 5 && kind <= 8)) &&
      kind == path_kind(pg.N, gflags) && !(flags & KBE_GREATER) && (gflags & KBE_INT_GREXTRA)) {
    if (kind == KIND_MFMA) launch_grad16(2, p, pg, p.n + 2 + p.ntau, st);
    else launch_grad8(2, p, pg, p.n + 2 + p.ntau, st);
  } else {
    vjp_grads(p, flags, st);
    vjp_grads(pg, gflags, st);
  }
  return hipGetLastError();
}


// ------------------------------------------------------------------------------------------
// Host-side audit of the work decomposition (a self-check, run on the CPU by the test-suite).
// For the plan a call would launch, it walks every task of every class the way the kernels do:
// the workgroup union of its outputs' term ranges clipped to the task's chunk (MFMA and
// small-block tasks, which stage the shared operand Q for every term of that union), or one
// output's range (generic tasks).  It checks that every staged Q block, and every weight and
// streamed block P of a term inside its output's own range, lies inside the array it is taken
// from.  Addresses are formed from distinct dummy base addresses and never dereferenced.
// ------------------------------------------------------------------------------------------
namespace {
struct AuditArr {
  uintptr_t base;
  int64_t count;  // elements
  int64_t esize;  // bytes per element
  bool in(const void *q) const {
    const uintptr_t a = (uintptr_t)q;
    if (a < base) return false;
    const uintptr_t d = a - base;
    return d % (uintptr_t)esize == 0 && (int64_t)(d / (uintptr_t)esize) < count;
  }
};

// CQ2 >= 0: the tasks also stage class CQ2's operand (from qa2) for every term of the union
// (a paired class, FusedPlan::pair).
template <int CLS, int CQ2 = -1>
void audit_class(const Params &p, const FusedPlan &pl, int k, int kind, const AuditArr *qa,
                 const AuditArr *const *pa, int npa, const AuditArr *wa, int nwa,
                 int64_t &bad, int64_t &checked, const AuditArr *qa2 = nullptr) {
  const int nch = pl.nchunk[k], nout = pl.nout[k], ngroup = pl.ngroup[k];
  const int64_t ntask = (int64_t)nch * ((ngroup + 3) / 4);
  for (int64_t lb = 0; lb < ntask; ++lb) {
    const int ch = (int)(lb % nch), gb = (int)(lb / nch);
    const int c0 = ch * pl.SC, c1 = c0 + pl.SC;
    int T0 = 1 << 30, T1 = 0;
    for (int wave = 0; wave < 4; ++wave) {
      const int g = gb * 4 + wave;
      if (g >= ngroup) continue;
      const int o0 = kind == KIND_GENERIC ? g : g * pl.MO;
      const int o1 = kind == KIND_GENERIC ? g + 1 : (o0 + pl.MO < nout ? o0 + pl.MO : nout);
      for (int o = o0; o < o1; ++o) {
        int lo, hi;
        cls_range<CLS>(p, o, lo, hi);
        if (kind == KIND_GENERIC) {  // one output per wave: only its own terms in this chunk
          const int a = lo > c0 ? lo : c0, b = hi < c1 ? hi : c1;
          for (int t = a; t < b; ++t) {
            ++checked;
            bad += !qa->in(cls_Q<CLS>(p, t));
          }
        } else {
          T0 = lo < T0 ? lo : T0;
          T1 = hi > T1 ? hi : T1;
        }
        const int a = lo > c0 ? lo : c0, b = hi < c1 ? hi : c1;
        for (int t = a; t < b; ++t) {  // weight and streamed block of each own term
          const double *w;
          const kbe_c128 *P;
          cls_wpP<CLS>(p, o, t, w, P);
          bool okP = false, okW = false;
          for (int i = 0; i < npa; ++i) okP = okP || pa[i]->in(P);
          for (int i = 0; i < nwa; ++i) okW = okW || wa[i].in(w);
          ++checked;
          bad += !(okP && okW);
        }
      }
    }
    if (kind != KIND_GENERIC) {  // the workgroup stages Q for every term of the union
      const int a = T0 > c0 ? T0 : c0, b = T1 < c1 ? T1 : c1;
      for (int t = a; t < b; ++t) {
        ++checked;
        bad += !qa->in(cls_Q<CLS>(p, t));
        if constexpr (CQ2 >= 0) {
          ++checked;
          bad += !qa2->in(cls_Q<CQ2>(p, t));
        }
      }
    }
  }
}
}  // namespace

}  // namespace kbe

// Declared in kbe_internal.h.
extern "C" int64_t kbe_internal_audit_tasks(int32_t N, int32_t nt, int32_t ntau, int64_t ldt,
                                            int32_t n, int32_t m0, int32_t m1, uint32_t flags,
                                            int32_t adjoint, int64_t *terms_checked) {
  using namespace kbe;
  const int kind = path_kind(N, flags);
  FusedPlan pl;
  if (adjoint) plan_adjoint(N, ntau, n, m0, m1, flags, kind, pl);
  else plan_forward(N, ntau, n, m0, m1, flags, kind, pl);
  const int64_t E = (int64_t)N * N, cs = sizeof(kbe_c128), ds = sizeof(double);
  const int M = m1 - m0;
  uintptr_t next = (uintptr_t)1 << 44;
  auto arr = [&](int64_t count, int64_t esize) {
    AuditArr a{next, count, esize};
    next += (uintptr_t)1 << 42;
    return a;
  };
  // the greater form's I^< reads a Sigma^> row of m1 blocks from the workspace
  const bool both = !adjoint && (flags & KBE_INT_BOTH);
  const bool sg = !adjoint && pl.sgoff >= 0 && !both;
  AuditArr kp = arr((int64_t)nt * ldt * E, cs), rdiag = arr((int64_t)nt * E, cs),
           tv = arr((int64_t)nt * ntau * E, cs), mat = arr((int64_t)ntau * E, cs),
           ret = arr((int64_t)(n + 1) * E, cs), les = arr((int64_t)(sg ? m1 : n + 1) * E, cs),
           stv = arr((int64_t)ntau * E, cs), w = arr((int64_t)nt * nt, ds),
           wtau = arr(ntau, ds), wf = arr((int64_t)ntau * ntau, ds),
           gIR = arr((int64_t)M * E, cs), gIL = arr((int64_t)M * E, cs),
           gItv = arr((int64_t)M * E, cs), gJ = arr((int64_t)ntau * E, cs),
           sgt = arr((int64_t)m1 * E, cs);
  // element-granular checks: kp and tv blocks are whole blocks, so count blocks as elements of
  // E complex numbers where a block start is what is formed
  AuditArr kpb{kp.base, (int64_t)nt * ldt, E * cs}, rdb{rdiag.base, nt, E * cs},
      tvb{tv.base, (int64_t)nt * ntau, E * cs}, matb{mat.base, ntau, E * cs},
      retb{ret.base, n + 1, E * cs}, lesb{les.base, sg ? m1 : n + 1, E * cs},
      stvb{stv.base, ntau, E * cs}, gIRb{gIR.base, M, E * cs}, gILb{gIL.base, M, E * cs},
      gItvb{gItv.base, M, E * cs}, gJb{gJ.base, ntau, E * cs}, sgtb{sgt.base, m1, E * cs};
  Params p{};
  p.N = N; p.nt = nt; p.ntau = ntau; p.J = ntau - 1; p.n = n; p.m0 = m0; p.m1 = m1; p.ldt = ldt;
  p.kp = (const kbe_c128 *)kp.base; p.rdiag = (const kbe_c128 *)rdiag.base;
  p.tv = (const kbe_c128 *)tv.base; p.mat = (const kbe_c128 *)mat.base;
  p.ret = (const kbe_c128 *)ret.base; p.les = (const kbe_c128 *)les.base;
  p.stv = (const kbe_c128 *)stv.base;
  p.sgt = both ? (const kbe_c128 *)sgt.base : nullptr;
  p.w = (const double *)w.base; p.wtau = (const double *)wtau.base; p.wf = (const double *)wf.base;
  p.gIR = (const kbe_c128 *)gIR.base; p.gIL = (const kbe_c128 *)gIL.base;
  p.gItv = (const kbe_c128 *)gItv.base; p.gJ = (const kbe_c128 *)gJ.base;
  const AuditArr *Pall[] = {&kpb, &rdb, &tvb, &matb, &gJb};
  const AuditArr Wall[] = {w, wtau, wf};
  int64_t bad = 0, checked = 0;
  for (int k = 0; k < pl.ncls; ++k) {
    const AuditArr *q = nullptr;
    switch (pl.cls[k]) {
      case C_IRC: case C_IRR: case C_JR: case C_GRL: case C_GRD: case C_GRU: q = &retb; break;
      case C_IL: q = &lesb; break;
      case C_ILX: q = &sgtb; break;
      case C_ITV: case C_JM1: case C_JM2: case G_MAT1: case G_MAT2: q = &stvb; break;
      case B_R1: case B_R2: case B_GRL: case B_GRD: case B_GRU: q = &gIRb; break;
      case B_L: case B_LGU: q = &gILb; break;
      case B_T1: q = &gItvb; break;
      default: q = &gJb; break;  // B_R3, B_T2A, B_T2B
    }
    if (pl.pair[k] >= 0) {  // C_GRU (B_GRU) on the tasks of C_IL, C_ILX (B_L); MFMA path
      const int pc = pl.cls[pl.pair[k]];
      if (pl.cls[k] == C_IL && pc == C_GRU)
        audit_class<C_IL, C_GRU>(p, pl, k, kind, q, Pall, 5, Wall, 3, bad, checked, &retb);
      else if (pl.cls[k] == C_ILX && pc == C_GRU)
        audit_class<C_ILX, C_GRU>(p, pl, k, kind, q, Pall, 5, Wall, 3, bad, checked, &retb);
      else if (pl.cls[k] == B_L && pc == B_GRU)
        audit_class<B_L, B_GRU>(p, pl, k, kind, q, Pall, 5, Wall, 3, bad, checked, &gIRb);
      else
        ++bad;
      continue;
    }
    switch (pl.cls[k]) {
#define KBE_CASE(C) \
  case C: audit_class<C>(p, pl, k, kind, q, Pall, 5, Wall, 3, bad, checked); break;
      KBE_CASE(C_IRC) KBE_CASE(C_IRR) KBE_CASE(C_IL) KBE_CASE(C_ITV) KBE_CASE(C_JR)
      KBE_CASE(C_JM1) KBE_CASE(C_JM2) KBE_CASE(B_R1) KBE_CASE(B_R2) KBE_CASE(B_R3) KBE_CASE(B_L)
      KBE_CASE(B_T1) KBE_CASE(B_T2A) KBE_CASE(B_T2B) KBE_CASE(G_MAT1) KBE_CASE(G_MAT2)
      KBE_CASE(C_GRL) KBE_CASE(C_GRD) KBE_CASE(C_GRU) KBE_CASE(B_GRL) KBE_CASE(B_GRD)
      KBE_CASE(B_GRU) KBE_CASE(C_ILX) KBE_CASE(B_LGU)
#undef KBE_CASE
      default: ++bad;
    }
  }
  (void)gItv;
  if (terms_checked) *terms_checked = checked;
  return bad;
}
