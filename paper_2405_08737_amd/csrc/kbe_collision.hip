// History integrals of arXiv:2405.08737 (Eq. KBE2 lesser form, history terms of Eq. KBE3) and
// their adjoint, on gfx950.
//
// Every output block is a sum of block products  c_t * Q_t * op(P_t)  over a list of terms t:
// P_t is a block of the (large) Green's-function storage streamed from HBM, Q_t a block of a
// (small, cache-resident) self-energy row or cotangent, c_t a scalar weight.  op is one of
//   OP_N : Q P        (contraction over P's row index)
//   OP_H : Q P^dagger (contraction over P's column index)
//   OP_HN: Q^dagger P
// Each family of terms ("class") enumerates its terms for an output index o.  The term list of
// an output is cut into chunks of SC terms; one wavefront computes one (output, chunk) partial
// sum and writes it to the workspace, and a reduce kernel adds the chunks in a fixed order, so
// results are deterministic (no floating-point atomics).
//
// Two implementations of the per-wave partial sum:
//   * stream_mfma16 (N = 16): FP64 matrix cores.  A 16x16 complex block product is 4 real
//     products, each 4 v_mfma_f64_16x16x4 over k-slices.  Operands are loaded straight from
//     global memory into the MFMA register layouts: the B operand (lane l holds B[k][l%16],
//     k = 4*slice + l/16) is a contiguous 1 KiB row-slice of a row-major block; the A operand
//     (lane l holds A[l%16][k]) reads 64-byte row segments.
//   * stream_generic (any N <= 16): vector ALU, one output element per lane, several terms per
//     wave for small N, lanes summed through LDS at the end.
#include "kbe_dev.h"
#include "kbe_internal.h"

#include <initializer_list>

namespace kbe {

enum Cls {
  C_IRC,   // I^R, column part: s <= m,  w[n][s] Sigma^R(n,s) G^<(s,m),       G^< = kp[s][m]
  C_IRR,   // I^R, row part:    s > m,  -w[n][s] Sigma^R(n,s) kp[m][s]^dagger
  C_IL,    // I^<:              s <= m,  w[m][s] Sigma^<(n,s) G^R(m,s)^dagger
  C_ITV,   // I^]:  -i wtau[j] Sigma^](n,j) tv[m][J-j]^dagger
  C_JR,    // J^] real-time part:  w[n][s] Sigma^R(n,s) tv[s][j]
  C_JM,    // J^] Matsubara part (split at tau_j)
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

template <int CLS>
__device__ __forceinline__ int cls_count(const Params &p, int o) {
  const int m = p.m0 + o;
  switch (CLS) {
    case C_IRC: return m + 1;
    case C_IRR: return p.n - m;
    case C_IL: return m + 1;
    case C_ITV: return p.ntau;
    case C_JR: return p.n + 1;
    case C_JM: return p.ntau + 1;
    case B_R1: { int lo = o > p.m0 ? o : p.m0; return p.m1 > lo ? p.m1 - lo : 0; }
    case B_R2: { int hi = o < p.m1 ? o : p.m1; return hi > p.m0 ? hi - p.m0 : 0; }
    case B_R3: return p.ntau;
    case B_L: { int lo = o > p.m0 ? o : p.m0; return p.m1 > lo ? p.m1 - lo : 0; }
    case B_T1: return p.m1 - p.m0;
    case B_T2: return p.ntau + 1;
    case G_MAT: return p.ntau + 1;
  }
  return 0;
}

// Term t of output o: scalar c, small operand Q, streamed block P.
template <int CLS>
__device__ __forceinline__ void cls_term(const Params &p, int o, int t, cd &c, const kbe_c128 *&Q,
                                         const kbe_c128 *&P) {
  const int64_t E = bsz(p);
  const int J = p.J;
  switch (CLS) {
    case C_IRC: {
      const int m = p.m0 + o, s = t;
      c = {p.w[(int64_t)p.n * p.nt + s], 0.0};
      Q = p.ret + s * E;
      P = kp_blk(p, s, m);
      break;
    }
    case C_IRR: {
      const int m = p.m0 + o, s = m + 1 + t;
      c = {-p.w[(int64_t)p.n * p.nt + s], 0.0};
      Q = p.ret + s * E;
      P = kp_blk(p, m, s);
      break;
    }
    case C_IL: {
      const int m = p.m0 + o, s = t;
      c = {p.w[(int64_t)m * p.nt + s], 0.0};
      Q = p.les + s * E;
      P = s < m ? kp_blk(p, m, s) : p.rdiag + m * E;
      break;
    }
    case C_ITV: {
      const int m = p.m0 + o, j = t;
      c = {0.0, -p.wtau[j]};
      Q = p.stv + j * E;
      P = tv_blk(p, m, J - j);
      break;
    }
    case C_JR: {
      const int s = t;
      c = {p.w[(int64_t)p.n * p.nt + s], 0.0};
      Q = p.ret + s * E;
      P = tv_blk(p, s, o);
      break;
    }
    case C_JM: {
      const int j = o;
      int l;
      if (t <= j) {  // [0, tau_j]: G^M(tau_l - tau_j) = -G^M(beta + tau_l - tau_j)
        l = t;
        c = {-p.wf[(int64_t)j * p.ntau + l], 0.0};
        P = p.mat + (J + l - j) * E;
      } else {       // [tau_j, beta]: mirror of the forward rule on the symmetric grid
        l = t - 1;
        c = {p.wf[(int64_t)(J - j) * p.ntau + (J - l)], 0.0};
        P = p.mat + (l - j) * E;
      }
      Q = p.stv + l * E;
      break;
    }
    case B_R1: {
      const int s = o, m = (s > p.m0 ? s : p.m0) + t;
      c = {p.w[(int64_t)p.n * p.nt + s], 0.0};
      Q = p.gIR + (m - p.m0) * E;
      P = kp_blk(p, s, m);
      break;
    }
    case B_R2: {
      const int s = o, m = p.m0 + t;
      c = {-p.w[(int64_t)p.n * p.nt + s], 0.0};
      Q = p.gIR + (m - p.m0) * E;
      P = kp_blk(p, m, s);
      break;
    }
    case B_R3: {
      const int s = o, j = t;
      c = {p.w[(int64_t)p.n * p.nt + s], 0.0};
      Q = p.gJ + j * E;
      P = tv_blk(p, s, j);
      break;
    }
    case B_L: {
      const int s = o, m = (s > p.m0 ? s : p.m0) + t;
      c = {p.w[(int64_t)m * p.nt + s], 0.0};
      Q = p.gIL + (m - p.m0) * E;
      P = m > s ? kp_blk(p, m, s) : p.rdiag + s * E;
      break;
    }
    case B_T1: {
      const int j = o, m = p.m0 + t;
      c = {0.0, p.wtau[j]};
      Q = p.gItv + t * E;
      P = tv_blk(p, m, J - j);
      break;
    }
    case B_T2: {
      const int l = o;
      int j;
      if (t < J - l + 1) {
        j = l + t;
        c = {-p.wf[(int64_t)j * p.ntau + l], 0.0};
        P = p.mat + (J + l - j) * E;
      } else {
        j = t - (J - l + 1);
        c = {p.wf[(int64_t)(J - j) * p.ntau + (J - l)], 0.0};
        P = p.mat + (l - j) * E;
      }
      Q = p.gJ + j * E;
      break;
    }
    case G_MAT: {
      const int k = o;
      int l, j;
      if (t <= k) {
        l = t;
        j = l + J - k;
        c = {-p.wf[(int64_t)j * p.ntau + l], 0.0};
      } else {
        j = t - (k + 1);
        l = j + k;
        c = {p.wf[(int64_t)(J - j) * p.ntau + (J - l)], 0.0};
      }
      Q = p.stv + l * E;
      P = p.gJ + j * E;
      break;
    }
  }
}

// Runtime dispatch of cls_count (used by the reduce to skip chunks past an output's last term).
__device__ __forceinline__ int count_rt(int cls, const Params &p, int o) {
  switch (cls) {
    case C_IRC: return cls_count<C_IRC>(p, o);
    case C_IRR: return cls_count<C_IRR>(p, o);
    case C_IL: return cls_count<C_IL>(p, o);
    case C_ITV: return cls_count<C_ITV>(p, o);
    case C_JR: return cls_count<C_JR>(p, o);
    case C_JM: return cls_count<C_JM>(p, o);
    case B_R1: return cls_count<B_R1>(p, o);
    case B_R2: return cls_count<B_R2>(p, o);
    case B_R3: return cls_count<B_R3>(p, o);
    case B_L: return cls_count<B_L>(p, o);
    case B_T1: return cls_count<B_T1>(p, o);
    case B_T2: return cls_count<B_T2>(p, o);
    case G_MAT: return cls_count<G_MAT>(p, o);
  }
  return 0;
}

// ------------------------------------------------------------------------------------------
// Generic vector-ALU partial sum of one (output, chunk) task by one wave.  For N*N <= 64 the
// wave runs G = 64/(N*N) groups of N*N lanes over interleaved terms (lane = one output
// element) and the groups are summed with cross-lane shuffles; for larger N each lane owns up
// to 4 elements.
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
      cd c;
      const kbe_c128 *Q, *P;
      cls_term<CLS>(p, o, t, c, Q, P);
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
// FP64 MFMA partial sum (N = 16).  Raw products are accumulated as
//   rr += A.re B.re, ii += A.im B.im, ri += A.re B.im, ir += A.im B.re
// with the A/B slots holding, per op (Q' = c Q, or conj(c) Q for OP_HN):
//   OP_N : A = Q'[l%16][k]   B = P[k][l%16]        -> D = Q'P:      (rr - ii, ri + ir)
//   OP_H : A = P[l%16][k]    B = Q'[l%16][k] (raw)  -> E = P Q'^dag: (rr + ii, ir - ri), out = E^dag
//   OP_HN: A = Q'[k][l%16]   B = P[k][l%16]   (raw) -> D = Q'^dag P: (rr + ii, ri - ir)
// with k = 4*slice + l/16.  D/E layout: lane l holds element (4*(l/16) + r, l%16), r = 0..3.
// ------------------------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int CLS>
__device__ __forceinline__ void task_mfma16(const Params &p, int o, int t0, int t1, kbe_c128 *out,
                                            int lane) {
  constexpr int OP = cls_op<CLS>();
  const int row = lane & 15, q = lane >> 4;
  v4d rr = {0, 0, 0, 0}, ii = rr, ri = rr, ir = rr;
  const int offA = row * 16 + q;  // element (row, 4*slice + q): + 4*slice
  const int offB = q * 16 + row;  // element (4*slice + q, row): + 64*slice
  for (int t = t0; t < t1; ++t) {
    cd c;
    const kbe_c128 *Q, *P;
    cls_term<CLS>(p, o, t, c, Q, P);
    cd a[4], b[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      if (OP == OP_N) {
        a[sl] = c * ld(Q + offA + 4 * sl);
        b[sl] = ld(P + offB + 64 * sl);
      } else if (OP == OP_H) {
        a[sl] = ld(P + offA + 4 * sl);
        b[sl] = c * ld(Q + offA + 4 * sl);
      } else {
        a[sl] = cj(c) * ld(Q + offB + 64 * sl);
        b[sl] = ld(P + offB + 64 * sl);
      }
    }
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      rr = mfma(a[sl].re, b[sl].re, rr);
      ii = mfma(a[sl].im, b[sl].im, ii);
      ri = mfma(a[sl].re, b[sl].im, ri);
      ir = mfma(a[sl].im, b[sl].re, ir);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * q + r;
    if (OP == OP_N) st(out + i * 16 + row, cd{rr[r] - ii[r], ri[r] + ir[r]});
    else if (OP == OP_H) st(out + row * 16 + i, cd{rr[r] + ii[r], ri[r] - ir[r]});
    else st(out + i * 16 + row, cd{rr[r] + ii[r], ri[r] - ir[r]});
  }
}

// One launch covers every class of a call: classes occupy consecutive ranges of the flat task
// index (task = wave), a class's tasks are (output, chunk) pairs with the chunk fastest.
struct FusedPlan {
  int ncls, SC;
  int cls[8], nout[8], nchunk[8];
  int64_t first[9];  // first task of each class; first[ncls] = total
  int64_t off[8];    // byte offset of each class's partials in the workspace
};

template <bool MFMA, int CLS>
__device__ __forceinline__ void run_task(const Params &p, const FusedPlan &pl, int k, int64_t loc,
                                         char *ws, int lane) {
  const int nch = pl.nchunk[k];
  const int o = (int)(loc / nch), ch = (int)(loc % nch);
  const int cnt = cls_count<CLS>(p, o);
  const int t0 = ch * pl.SC;
  if (t0 >= cnt) return;  // empty chunk: nothing written, the reduce skips it
  const int t1 = cnt < t0 + pl.SC ? cnt : t0 + pl.SC;
  kbe_c128 *out = (kbe_c128 *)(ws + pl.off[k]) + ((int64_t)ch * pl.nout[k] + o) * bsz(p);
  if (MFMA) task_mfma16<CLS>(p, o, t0, t1, out, lane);
  else task_generic<CLS>(p, o, t0, t1, out, lane);
}

template <bool MFMA>
__global__ void __launch_bounds__(256) stream_fused(Params p, FusedPlan pl, char *ws) {
  const int lane = threadIdx.x & 63;
  const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (task >= pl.first[pl.ncls]) return;  // no block-level barriers anywhere below
  int k = 0;
  while (task >= pl.first[k + 1]) ++k;
  const int64_t loc = task - pl.first[k];
  switch (pl.cls[k]) {
    case C_IRC: run_task<MFMA, C_IRC>(p, pl, k, loc, ws, lane); break;
    case C_IRR: run_task<MFMA, C_IRR>(p, pl, k, loc, ws, lane); break;
    case C_IL: run_task<MFMA, C_IL>(p, pl, k, loc, ws, lane); break;
    case C_ITV: run_task<MFMA, C_ITV>(p, pl, k, loc, ws, lane); break;
    case C_JR: run_task<MFMA, C_JR>(p, pl, k, loc, ws, lane); break;
    case C_JM: run_task<MFMA, C_JM>(p, pl, k, loc, ws, lane); break;
    case B_R1: run_task<MFMA, B_R1>(p, pl, k, loc, ws, lane); break;
    case B_R2: run_task<MFMA, B_R2>(p, pl, k, loc, ws, lane); break;
    case B_R3: run_task<MFMA, B_R3>(p, pl, k, loc, ws, lane); break;
    case B_L: run_task<MFMA, B_L>(p, pl, k, loc, ws, lane); break;
    case B_T1: run_task<MFMA, B_T1>(p, pl, k, loc, ws, lane); break;
    case B_T2: run_task<MFMA, B_T2>(p, pl, k, loc, ws, lane); break;
    case G_MAT: run_task<MFMA, G_MAT>(p, pl, k, loc, ws, lane); break;
  }
}

// out[x] (=|+=) the sum, in increasing chunk order, of the non-empty chunks of up to three
// classes' partial arrays (chunk c of output o is non-empty when c*SC < count(o)).
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
    const int cnt = count_rt(in.cls[k], p, o);
    int nc = (cnt + in.SC - 1) / in.SC;
    if (nc > in.nchunk[k]) nc = in.nchunk[k];
    for (int c = 0; c < nc; ++c) s = s + ld(in.a[k] + (int64_t)c * nel + x);
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
    kbe_c128 *d = dst + (4 * q + r) * 16 + row;
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

// Add class cls with nout outputs of at most maxcnt terms to the plan (skipped when empty).
static void plan_add(FusedPlan &pl, int cls, int nout, int maxcnt, int E, size_t &off) {
  if (nout <= 0 || maxcnt <= 0) return;
  const int k = pl.ncls++;
  pl.cls[k] = cls;
  pl.nout[k] = nout;
  pl.nchunk[k] = (maxcnt + pl.SC - 1) / pl.SC;
  pl.off[k] = (int64_t)off;
  pl.first[k + 1] = pl.first[k] + (int64_t)nout * pl.nchunk[k];
  off += al256(sizeof(kbe_c128) * (size_t)pl.nchunk[k] * nout * E);
}

static FusedPlan plan_init(int N, bool mfma) {
  FusedPlan pl{};
  pl.SC = chunk_terms(N, mfma);
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
    plan_add(pl, C_IRR, M, n - m0, E, off);
  }
  if (flags & KBE_OUT_IL) plan_add(pl, C_IL, M, m1, E, off);
  if ((flags & KBE_OUT_ITV) && th) plan_add(pl, C_ITV, M, ntau, E, off);
  if ((flags & KBE_OUT_JTV) && th) {
    plan_add(pl, C_JR, ntau, n + 1, E, off);
    plan_add(pl, C_JM, ntau, ntau + 1, E, off);
  }
  return off;
}

static size_t plan_adjoint(int N, int ntau, int n, int m0, int m1, unsigned flags, bool mfma,
                           FusedPlan &pl) {
  pl = plan_init(N, mfma);
  const int E = N * N, M = m1 - m0;
  size_t off = 0;
  const bool th = ntau > 0;
  const bool fITV = (flags & KBE_OUT_ITV) && th, fJTV = (flags & KBE_OUT_JTV) && th;
  if (flags & KBE_OUT_IR) {
    plan_add(pl, B_R1, n + 1, M, E, off);
    plan_add(pl, B_R2, n + 1, M, E, off);
  }
  if (fJTV) plan_add(pl, B_R3, n + 1, ntau, E, off);
  if (flags & KBE_OUT_IL) plan_add(pl, B_L, n + 1, M, E, off);
  if (fITV) plan_add(pl, B_T1, ntau, M, E, off);
  if (fJTV) {
    plan_add(pl, B_T2, ntau, ntau + 1, E, off);
    plan_add(pl, G_MAT, ntau, ntau + 1, E, off);
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
  const int64_t tasks = pl.first[pl.ncls];
  if (tasks == 0) return;
  const dim3 grid((unsigned)((tasks + 3) / 4)), block(256);
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
