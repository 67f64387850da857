// Batches of history rows (the integrals of Eq. KBE2 at single (t_n, t_m) points of many
// independent systems), one persistent launch per call.
//
// Work unit ("task"): one wave sums one chunk of terms of one term class of one item:
//   IRC: s in [0, m]      wn[s] sig_ret[s] col[s]                      (Q P)
//   IRR: s in (m, n]     -wn[s] sig_ret[s] row[s]^dagger               (Q P^dagger)
//   IL : s in [0, m]      wm[s] sig_les[s] (row[s] | rdiag)^dagger     (Q P^dagger)
//   ITV: j in [0, ntau)  -i wtau[j] sig_tv[j] tv[J-j]^dagger           (Q P^dagger)
// Both factors of a term are streamed (nothing is shared between terms), so the work is bound by
// HBM bandwidth at every N (N/4 FLOP per byte).  Each wave takes tasks from one atomic counter
// and runs the code path of its item's N: one lane per term on the vector ALU (N <= 4), or
// blocks zero-padded to 8 x 8 (5 <= N <= 8) or 16 x 16 (9 <= N <= 16) multiplied with
// v_mfma_f64_4x4x4, three real products per complex one:
//   k1 += (ar + ai) br,  k2 += ar (bi - br),  k3 += ai (br + bi);  Re = k1 - k3, Im = k1 + k2.
// A task writes its partial sum to the workspace; a reduce adds an item's partials in task
// order, so results are deterministic.  The task plan (per-item task and partial offsets) is
// computed on the device from the item array, so a call copies nothing from host memory; it
// hands out the tasks of the largest blocks first.
#include "kbe_dev.h"
#include "kbe_internal.h"

namespace kbe {

namespace {

constexpr int BQLD = 20;     // LDS row stride of a staged 16 x 16 block, in complex numbers
constexpr int TB_LDS = 2048;  // task-offset entries kept in LDS (batches of up to 2047 items)

__device__ __forceinline__ double mfma4b(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int cdivd(int a, int b) { return (a + b - 1) / b; }

// A copy of *p held in scalar registers (p and *p the same for every lane of the wave), so that
// values and branches derived from it are wave-uniform.
template <typename T>
__device__ __forceinline__ T uniform_copy(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized struct");
  T v;
  const unsigned *src = (const unsigned *)p;
  unsigned *dst = (unsigned *)&v;
#pragma unroll
  for (int w = 0; w < (int)(sizeof(T) / 4); ++w) dst[w] = __builtin_amdgcn_readfirstlane(src[w]);
  return v;
}

// A double through a pointer known to address global memory (not a flat access).
__device__ __forceinline__ double ldgd(const double *p) {
  return *(const __attribute__((address_space(1))) double *)(const void *)p;
}

typedef double __attribute__((ext_vector_type(4))) d4b;
__device__ __forceinline__ d4b mfma16b(double a, double b, d4b c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Terms per work unit of an item: the call's chunk when it is set, else the item's own, else the
// default.
__host__ __device__ inline int item_chunk(const kbe_batch_item &it, int chunk) {
  return chunk > 0 ? chunk : it.chunk > 0 ? it.chunk : 64;
}

// Chunks per term class of an item: IRC, IRR, IL, ITV.
__host__ __device__ inline void item_chunks(const kbe_batch_item &it, int call_chunk, int c[4]) {
  const int chunk = item_chunk(it, call_chunk);
  const bool ir = it.flags & KBE_OUT_IR, il = it.flags & KBE_OUT_IL;
  const bool itv = (it.flags & KBE_OUT_ITV) && it.ntau > 0;
  c[0] = ir ? (it.m + 1 + chunk - 1) / chunk : 0;
  c[1] = ir ? (it.n - it.m + chunk - 1) / chunk : 0;
  c[2] = il ? (it.m + 1 + chunk - 1) / chunk : 0;
  c[3] = itv ? (it.ntau + chunk - 1) / chunk : 0;
}

// Blocks from col[s] to col[s+1] (a contiguous array, or a column of a KP storage read in place).
__host__ __device__ inline int64_t col_step(const kbe_batch_item &it) {
  return it.col_ld > 1 ? it.col_ld : 1;
}

// Term t of class k of an item: real weight w, complex factor (fr + i fi), Q and P blocks.
struct Term {
  double w;
  const kbe_c128 *Q, *P;
};
__device__ __forceinline__ Term item_term(const kbe_batch_item &it, int k, int t) {
  const int64_t E = (int64_t)it.N * it.N;
  switch (k) {
    case 0: return {it.wn[t], it.sig_ret + t * E, it.col + t * col_step(it) * E};
    case 1: return {it.wn[t], it.sig_ret + t * E, it.row + t * E};
    case 2: return {it.wm[t], it.sig_les + t * E, t < it.m ? it.row + t * E : it.rdiag};
    default: return {it.wtau[t], it.sig_tv + t * E, it.tv + (it.ntau - 1 - t) * E};
  }
}

// Term range [lo, hi) of class k.
__device__ __forceinline__ void item_range(const kbe_batch_item &it, int k, int &lo, int &hi) {
  switch (k) {
    case 0: lo = 0; hi = it.m + 1; break;
    case 1: lo = it.m + 1; hi = it.n + 1; break;
    case 2: lo = 0; hi = it.m + 1; break;
    default: lo = 0; hi = it.ntau; break;
  }
}

// Adjoint classes: the gradient blocks of a row, grouped by the product that gives them.
//   V0 g_sig_ret[s], s <= m:  wn[s] GR col[s]^dagger          (form GX^dagger)
//   V1 g_sig_ret[s], s > m : -wn[s] GR row[s]                  (form GX)
//   V2 g_sig_les[s], s <= m:  wm[s] GL (row[s] | rdiag)        (form GX)
//   V3 g_sig_les[s], s > m :  0
//   V4 g_col[s],     s <= m:  wn[s] sig_ret[s]^dagger GR       (form X^dagger G)
//   V5 g_row[s],     s > m : -wn[s] GR^dagger sig_ret[s]       (form G^dagger X)
//   V6 g_row[s],     s <= m:  wm[s] GL^dagger sig_les[s] (s < m), 0 (s = m)
//   V7 g_rdiag:               wm[m] GL^dagger sig_les[m]
//   V8 g_sig_tv[j]:           i wtau[j] GT tv[J-j]             (form GX)
//   V9 g_tv[k]:              -i wtau[J-k] GT^dagger sig_tv[J-k]
constexpr int VJP_CLASSES = 10;
// Output blocks per adjoint task: 64 at N > 4; more for smaller blocks, so that a task is a few
// steps of the vector-ALU loop rather than one (8 steps at N = 2, 4 and 8).
__host__ __device__ inline int vjp_chunk(int N) { return N <= 2 ? 1024 : (N <= 4 ? 256 : 64); }
constexpr int VJP_R = 2;       // blocks per thread per step of the adjoint (loads in flight)
enum VjpForm { F_GXH, F_GX, F_XHG, F_GHX, F_ZERO };

__host__ __device__ inline void vjp_range(const kbe_batch_item &r, int k, int &lo, int &hi) {
  switch (k) {
    case 0: case 2: case 4: case 6: lo = 0; hi = r.m + 1; break;
    case 1: case 3: case 5: lo = r.m + 1; hi = r.n + 1; break;
    case 7: lo = 0; hi = 1; break;
    default: lo = 0; hi = r.ntau; break;
  }
}

__host__ __device__ inline void vjp_chunks(const kbe_batch_item &r, int c[VJP_CLASSES]) {
  for (int k = 0; k < VJP_CLASSES; ++k) {
    int lo, hi;
    vjp_range(r, k, lo, hi);
    const int ch = vjp_chunk(r.N);
    c[k] = (hi - lo + ch - 1) / ch;
  }
}

// c = (fr + i fi) w per class: IRC 1, IRR -1, IL 1, ITV -i.
__device__ __forceinline__ cd class_factor(int k, double w) {
  return k == 1 ? cd{-w, 0.0} : (k == 3 ? cd{0.0, -w} : cd{w, 0.0});
}

// ---------------------------------------------------------------------------------------
// N <= 4: one lane per term, 64 terms per pass; the lane adds c Q op(P) into its N x N
// accumulator (op(P) = P or P^dagger), then the wave's 64 accumulators are summed by a
// reduce-scatter (the accumulator padded to EP = 1, 4 or 16 entries: halving steps on lane bits
// 5, 4, ... leave lane l with one entry, whose index is read from those bits, and the remaining
// lane bits are summed by butterflies).
// ---------------------------------------------------------------------------------------
template <int N>
__device__ void task_tiny(const kbe_batch_item &it, int k, int t0, int t1, kbe_c128 *out,
                          int lane) {
  constexpr int E = N * N, EP = E == 1 ? 1 : (E <= 4 ? 4 : 16), LB = EP == 1 ? 0 : (EP == 4 ? 2 : 4);
  const bool dag = k != 0;
  cd acc[EP];
#pragma unroll
  for (int e = 0; e < EP; ++e) acc[e] = czero();
  for (int t = t0 + lane; t < t1; t += 64) {
    const Term tm = item_term(it, k, t);
    const cd c = class_factor(k, tm.w);
    cd q[E], p[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      q[e] = ldg(tm.Q + e);
      p[e] = ldg(tm.P + e);
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int l = 0; l < N; ++l) {
        const cd cq = c * q[i * N + l];
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const cd x = dag ? cj(p[j * N + l]) : p[l * N + j];
          cd &a = acc[i * N + j];
          a.re = __builtin_fma(cq.re, x.re, a.re);
          a.re = __builtin_fma(-cq.im, x.im, a.re);
          a.im = __builtin_fma(cq.re, x.im, a.im);
          a.im = __builtin_fma(cq.im, x.re, a.im);
        }
      }
  }
#pragma unroll
  for (int s = 0; s < LB; ++s) {
    const int m = 32 >> s, c = EP >> (s + 1);
    const bool up = lane & m;
#pragma unroll
    for (int kk = 0; kk < c; ++kk) {
      const cd lo = acc[kk], hi = acc[kk + c];
      const cd send = up ? lo : hi, keep = up ? hi : lo;
      acc[kk].re = keep.re + __shfl_xor(send.re, m);
      acc[kk].im = keep.im + __shfl_xor(send.im, m);
    }
  }
#pragma unroll
  for (int m = 32 >> LB; m >= 1; m >>= 1) {
    acc[0].re += __shfl_xor(acc[0].re, m);
    acc[0].im += __shfl_xor(acc[0].im, m);
  }
  int e = 0;
#pragma unroll
  for (int s = 0; s < LB; ++s) e = (e << 1) | ((lane >> (5 - s)) & 1);
  if ((lane & ((64 >> LB) - 1)) == 0 && e < E) stg(out + e, acc[0]);
}

// ---------------------------------------------------------------------------------------
// N <= 8: blocks padded to 8 x 8; one instruction computes the four 4 x 4 tiles (ti, tj) of the
// product (instruction block b = 2 ti + tj).  Lane roles: A element (4ti + lj, 4kc + lk) of
// c Q, B element (4kc + lk, 4tj + lj) of P, or conj of P's (4tj + lj, 4kc + lk) for P^dagger,
// D element (4ti + lk, 4tj + lj).  Terms are loaded three ahead of their use.
// ---------------------------------------------------------------------------------------
__device__ void task8(const kbe_batch_item &it, int k, int t0, int t1, kbe_c128 *out, int lane) {
  const int N = it.N;
  const bool dag = k != 0;
  const int lj = lane & 3, lk = lane >> 4, tb = (lane >> 2) & 3, ti = tb >> 1, tj = tb & 1;
  bool av[2], bv[2];
  int ao[2], bo[2];
#pragma unroll
  for (int kc = 0; kc < 2; ++kc) {
    const int ra = 4 * ti + lj, ca = 4 * kc + lk;
    av[kc] = ra < N && ca < N;
    ao[kc] = av[kc] ? ra * N + ca : 0;
    const int rb = dag ? 4 * tj + lj : 4 * kc + lk, cb = dag ? 4 * kc + lk : 4 * tj + lj;
    bv[kc] = rb < N && cb < N;
    bo[kc] = bv[kc] ? rb * N + cb : 0;
  }
  struct Buf {
    double w;
    cd q[2], x[2];
  };
  auto load = [&](int t, Buf &b) {
    t = t < t1 ? t : t1 - 1;
    const Term tm = item_term(it, k, t);
    b.w = tm.w;
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      b.q[kc] = ldg(tm.Q + ao[kc]);
      b.x[kc] = ldg(tm.P + bo[kc]);
    }
  };
  double k1 = 0.0, k2 = 0.0, k3 = 0.0;
  auto compute = [&](const Buf &b) {
    const cd c = class_factor(k, b.w);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const cd q = av[kc] ? c * b.q[kc] : czero();
      cd x = bv[kc] ? b.x[kc] : czero();
      if (dag) x.im = -x.im;
      k1 = mfma4b(q.re + q.im, x.re, k1);
      k2 = mfma4b(q.re, x.im - x.re, k2);
      k3 = mfma4b(q.im, x.re + x.im, k3);
    }
  };
  Buf bf[4];
  load(t0, bf[0]);
  load(t0 + 1, bf[1]);
  load(t0 + 2, bf[2]);
  for (int t = t0; t < t1; t += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (t + u >= t1) break;  // wave-uniform
      load(t + u + 3, bf[(u + 3) & 3]);
      __builtin_amdgcn_sched_barrier(0);
      compute(bf[u]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const int dr = 4 * ti + lk, dc = 4 * tj + lj;
  if (dr < N && dc < N) stg(out + dr * N + dc, cd{k1 - k3, k1 + k2});
}

// ---------------------------------------------------------------------------------------
// N = 16: v_mfma_f64_16x16x4 with both operands loaded straight into their lane layouts, no
// LDS: lane l supplies A[l%16][4kc + l/16] = c Q[l%16][4kc + l/16] and B[4kc + l/16][l%16], which
// is P[4kc + l/16][l%16] (Q P) or conj P[l%16][4kc + l/16] (Q P^dagger), and holds
// D[l/16 + 4r][l%16].  Three real products per complex one; three terms in flight.
// ---------------------------------------------------------------------------------------
__device__ void task16d(const kbe_batch_item &it, int k, int t0, int t1, kbe_c128 *out,
                        int lane) {
  const bool dag = k != 0;
  const int lk = lane >> 4, lc = lane & 15;
  struct Buf {
    double w;
    cd q[4], x[4];
  };
  auto load = [&](int t, Buf &b) {
    t = t < t1 ? t : t1 - 1;
    const Term tm = item_term(it, k, t);
    b.w = tm.w;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      b.q[kc] = ldg(tm.Q + lc * 16 + 4 * kc + lk);
      b.x[kc] = ldg(tm.P + (dag ? lc * 16 + 4 * kc + lk : (4 * kc + lk) * 16 + lc));
    }
  };
  d4b k1 = {0, 0, 0, 0}, k2 = {0, 0, 0, 0}, k3 = {0, 0, 0, 0};
  auto compute = [&](const Buf &b) {
    const cd c = class_factor(k, b.w);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const cd a = c * b.q[kc];
      cd x = b.x[kc];
      if (dag) x.im = -x.im;
      k1 = mfma16b(a.re + a.im, x.re, k1);
      k2 = mfma16b(a.re, x.im - x.re, k2);
      k3 = mfma16b(a.im, x.re + x.im, k3);
    }
  };
  Buf b0, b1, b2;
  load(t0, b0);
  load(t0 + 1, b1);
  for (int t = t0; t < t1; t += 3) {
    load(t + 2, b2);
    __builtin_amdgcn_sched_barrier(0);
    compute(b0);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 >= t1) break;  // wave-uniform
    load(t + 3, b0);
    __builtin_amdgcn_sched_barrier(0);
    compute(b1);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 2 >= t1) break;
    load(t + 4, b1);
    __builtin_amdgcn_sched_barrier(0);
    compute(b2);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) stg(out + (lk + 4 * r) * 16 + lc, cd{k1[r] - k3[r], k1[r] + k2[r]});
}

// ---------------------------------------------------------------------------------------
// 9 <= N <= 16: blocks padded to 16 x 16, the layout of the N = 16 collision task: the wave
// stages c Q in its own LDS tile (rows padded to BQLD complex numbers), lane l supplies
// A[4ti + l%4][4kc + l/16] from it and the slab B[4kc + l/16][l%16] of P (or P^dagger), and
// accumulator ti holds D[4ti + l/16][l%16].  The next two terms' Q and P are in flight during a
// term's products.
// ---------------------------------------------------------------------------------------
__device__ void task16(const kbe_batch_item &it, int k, int t0, int t1, kbe_c128 *out, int lane,
                       cd *qs) {
  const int N = it.N;
  const bool dag = k != 0;
  const int lr = lane & 3, lk = lane >> 4, lc = lane & 15;
  int qo[4], bo[4];
  bool qv[4], bv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = lane + 64 * u, r = e >> 4, c = e & 15;  // Q element staged by this lane
    qv[u] = r < N && c < N;
    qo[u] = qv[u] ? r * N + c : 0;
    const int rb = dag ? lc : 4 * u + lk, cb = dag ? 4 * u + lk : lc;  // B slab u element
    bv[u] = rb < N && cb < N;
    bo[u] = bv[u] ? rb * N + cb : 0;
  }
  struct Buf {
    double w;
    cd q[4], x[4];
  };
  auto load = [&](int t, Buf &b) {
    t = t < t1 ? t : t1 - 1;
    const Term tm = item_term(it, k, t);
    b.w = tm.w;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      b.q[u] = ldg(tm.Q + qo[u]);
      b.x[u] = ldg(tm.P + bo[u]);
    }
  };
  double k1[4] = {0, 0, 0, 0}, k2[4] = {0, 0, 0, 0}, k3[4] = {0, 0, 0, 0};
  auto compute = [&](const Buf &b) {
    const cd c = class_factor(k, b.w);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = lane + 64 * u;
      qs[(e >> 4) * BQLD + (e & 15)] = qv[u] ? c * b.q[u] : czero();
    }
    // the wave's own LDS writes are complete before its reads (in-order LDS queue); the
    // compiler keeps the order since the accesses may alias
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      cd x = bv[kc] ? b.x[kc] : czero();
      if (dag) x.im = -x.im;
      const double br = x.re, bd = x.im - x.re, bp = x.re + x.im;
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) {
        const cd a = qs[(4 * ti + lr) * BQLD + 4 * kc + lk];
        k1[ti] = mfma4b(a.re + a.im, br, k1[ti]);
        k2[ti] = mfma4b(a.re, bd, k2[ti]);
        k3[ti] = mfma4b(a.im, bp, k3[ti]);
      }
    }
  };
  Buf b0, b1, b2;  // two terms in flight
  load(t0, b0);
  load(t0 + 1, b1);
  for (int t = t0; t < t1; t += 3) {
    load(t + 2, b2);
    __builtin_amdgcn_sched_barrier(0);
    compute(b0);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 >= t1) break;  // wave-uniform
    load(t + 3, b0);
    __builtin_amdgcn_sched_barrier(0);
    compute(b1);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 2 >= t1) break;
    load(t + 4, b1);
    __builtin_amdgcn_sched_barrier(0);
    compute(b2);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int ti = 0; ti < 4; ++ti) {
    const int r = 4 * ti + lk;
    if (r < N && lc < N) stg(out + r * N + lc, cd{k1[ti] - k3[ti], k1[ti] + k2[ti]});
  }
}

}  // namespace

// Plan (one workgroup of 1024 threads):
//   perm[count]  processing order: items by decreasing N, stable (the heaviest tasks are taken
//                first, so the launch does not end on a tail of large blocks; results do not
//                depend on the order, since each item's partials are laid out and summed by
//                chunk index);
//   tb[count+1]  task offsets in that order (exclusive scan);
//   pb[count+1]  partial offsets in item order, in complex numbers (exclusive scan);
// and zeroes the task counter.
// Inclusive scan over the 1024 threads of the workgroup (wave shuffles, then the 16 wave totals);
// every thread calls it; *total receives the sum.  ws: 16 shared slots.
__device__ __forceinline__ int64_t block_scan(int64_t v, int64_t *ws, int64_t *total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  if (lane == 63) ws[w] = v;
  __syncthreads();
  if (w == 0) {
    int64_t x = lane < 16 ? ws[lane] : 0;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int64_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane < 16) ws[lane] = x;
  }
  __syncthreads();
  v += w > 0 ? ws[w - 1] : 0;
  *total = ws[15];
  __syncthreads();  // ws is reused by the next scan
  return v;
}

// Per-item task and partial counts of the forward (partials: one N x N block per task) and of
// the adjoint (tasks of vjp_chunk(N) output blocks, no partials).
__device__ inline const kbe_batch_item &row_of(const kbe_batch_item &x) { return x; }
__device__ inline const kbe_batch_item &row_of(const kbe_batch_vjp_item &x) { return x.row; }
__device__ inline int64_t plan_tasks(const kbe_batch_item &it, int chunk) {
  int c[4];
  item_chunks(it, chunk, c);
  return c[0] + c[1] + c[2] + c[3];
}
__device__ inline int64_t plan_parts(const kbe_batch_item &it, int chunk) {
  return plan_tasks(it, chunk) * it.N * it.N;
}
__device__ inline int64_t plan_tasks(const kbe_batch_vjp_item &it, int) {
  int c[VJP_CLASSES];
  vjp_chunks(it.row, c);
  int64_t t = 0;
#pragma unroll
  for (int k = 0; k < VJP_CLASSES; ++k) t += c[k];
  return t;
}
__device__ inline int64_t plan_parts(const kbe_batch_vjp_item &, int) { return 0; }

template <typename Item>
__global__ void __launch_bounds__(1024) batch_plan(const Item *items, int count, int chunk,
                                                   int *perm, int64_t *tb, int64_t *pb,
                                                   unsigned int *head) {
  __shared__ int64_t wsum[16];
  __shared__ int nbin[KBE_NMAX + 1];
  const int tid = threadIdx.x;
  if (tid <= KBE_NMAX) nbin[tid] = 0;
  __syncthreads();
  for (int i = tid; i < count; i += 1024) atomicAdd(&nbin[row_of(items[i]).N], 1);  // integer counts
  __syncthreads();
  // stable counting sort, N from KBE_NMAX down to 1 (empty bins skipped)
  int64_t placed = 0;
  for (int N = KBE_NMAX; N >= 1; --N) {
    if (nbin[N] == 0) continue;  // uniform
    for (int base = 0; base < count; base += 1024) {
      const int i = base + tid;
      const int64_t hit = i < count && row_of(items[i]).N == N;
      int64_t tot;
      const int64_t r = block_scan(hit, wsum, &tot);
      if (hit) perm[placed + r - 1] = i;
      placed += tot;
    }
  }
  __syncthreads();  // perm (global memory, written by other threads) is read below
  // task offsets in processing order, partial offsets in item order
  int64_t carry_t = 0, carry_p = 0;
  for (int base = 0; base < count; base += 1024) {
    const int j = base + tid;
    int64_t nt = 0, np = 0;
    if (j < count) {
      nt = plan_tasks(items[perm[j]], chunk);
      np = plan_parts(items[j], chunk);
    }
    int64_t tt, tp;
    const int64_t st = block_scan(nt, wsum, &tt);
    const int64_t sp = block_scan(np, wsum, &tp);
    if (j < count) {
      tb[j] = carry_t + st - nt;
      pb[j] = carry_p + sp - np;
    }
    carry_t += tt;
    carry_p += tp;
  }
  if (tid == 0) {
    tb[count] = carry_t;
    pb[count] = carry_p;
    head[0] = 0u;
  }
}

// Persistent: every wave takes tasks from the counter until none are left.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) batch_stream(const kbe_batch_item *items, int count,
                                                    int chunk, const int *perm,
                                                    const int64_t *tb, const int64_t *pb,
                                                    kbe_c128 *parts, unsigned int *head) {
  __shared__ cd qtile[4][16 * BQLD];
  __shared__ int64_t tbs[TB_LDS];  // the task offsets, when they fit
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool cached = count < TB_LDS;  // uniform
  if (cached)
    for (int j = threadIdx.x; j <= count; j += blockDim.x) tbs[j] = tb[j];
  __syncthreads();
  const int64_t ntask = tb[count];
  for (;;) {
    unsigned int v = 0;
    if (lane == 0) v = atomicAdd(head, 1u);
    const int64_t task = (int64_t)__builtin_amdgcn_readfirstlane(v);
    if (task >= ntask) break;  // wave-uniform
    // position in the processing order: the last j with tb[j] <= task (binary search, in LDS
    // when the table fits)
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((cached ? tbs[mid] : tb[mid]) <= task) lo = mid;
      else hi = mid - 1;
    }
    const int j = __builtin_amdgcn_readfirstlane(lo);
    const int i = __builtin_amdgcn_readfirstlane(perm[j]);
    const kbe_batch_item it = items[i];
    int c[4];
    item_chunks(it, chunk, c);
    // (an LDS read: made wave-uniform explicitly, so that the task's ranges and loops are)
    const int64_t ltask =
        (int64_t)__builtin_amdgcn_readfirstlane((int)(task - (cached ? tbs[j] : tb[j])));
    int local = (int)ltask, k = 0;
    while (local >= c[k]) local -= c[k++];
    int t0, t1;
    item_range(it, k, t0, t1);
    const int ch = item_chunk(it, chunk);
    t0 += local * ch;
    t1 = t0 + ch < t1 ? t0 + ch : t1;
    kbe_c128 *out = parts + pb[i] + ltask * (int64_t)it.N * it.N;
    switch (it.N) {  // wave-uniform
      case 1: task_tiny<1>(it, k, t0, t1, out, lane); break;
      case 2: task_tiny<2>(it, k, t0, t1, out, lane); break;
      case 3: task_tiny<3>(it, k, t0, t1, out, lane); break;
      case 4: task_tiny<4>(it, k, t0, t1, out, lane); break;
      default:
        if (it.N <= 8) task8(it, k, t0, t1, out, lane);
        else if (it.N == 16) task16d(it, k, t0, t1, out, lane);
        else task16(it, k, t0, t1, out, lane, qtile[wave]);
    }
  }
}

// One workgroup per item: element e of each selected output = its tasks' partials in order.
__global__ void __launch_bounds__(256) batch_reduce(const kbe_batch_item *items, int chunk,
                                                    const int64_t *pb, const kbe_c128 *parts) {
  const kbe_batch_item it = items[blockIdx.x];
  const int E = it.N * it.N, e = threadIdx.x;
  if (e >= E) return;
  int c[4];
  item_chunks(it, chunk, c);
  const kbe_c128 *p = parts + pb[blockIdx.x] + e;
  auto sum = [&](int a, int b) {  // eight loads in flight; added in chunk order
    cd s = czero();
    for (int L = a; L < b; L += 8) {
      cd v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = L + u < b ? ldg(p + (int64_t)(L + u) * E) : czero();
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (L + u < b) s = s + v[u];
    }
    return s;
  };
  const int irb = c[0] + c[1], ilb = irb + c[2], itb = ilb + c[3];
  if (it.flags & KBE_OUT_IR) stg(it.IR + e, sum(0, irb));
  if (it.flags & KBE_OUT_IL) stg(it.IL + e, sum(irb, ilb));
  if (it.flags & KBE_OUT_ITV) stg(it.Itv + e, sum(ilb, itb));
}

// Adjoint: persistent workgroups take tasks (item, class, up to vjp_chunk(N) output blocks) from one
// counter.  Blocks of one class go through in steps of VJP_R * 256 / EP blocks (EP = N^2 rounded
// up to a power of two); thread (block b, element e = i N + j) computes element (i, j) of its
// VJP_R output blocks from the cotangent's row or column (in registers for the whole task) and
// the streamed blocks X (staged in LDS, double-buffered, the next step's elements loaded ahead).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) batch_vjp_stream(const kbe_batch_vjp_item *items,
                                                        int count, const int *perm,
                                                        const int64_t *tb, unsigned int *head) {
  __shared__ int64_t tbs[TB_LDS];
  __shared__ cd xs[2][VJP_R * 256];
  __shared__ int64_t task_s;
  const int tid = threadIdx.x;
  const bool cached = count < TB_LDS;
  if (cached)
    for (int j = tid; j <= count; j += blockDim.x) tbs[j] = tb[j];
  __syncthreads();
  const int64_t ntask = tb[count];
  for (;;) {
    if (tid == 0) task_s = (int64_t)atomicAdd(head, 1u);
    __syncthreads();
    // (read through LDS; made wave-uniform explicitly so that everything derived from the task
    // stays in scalar registers and branches on it are uniform)
    const int64_t task = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((unsigned)task_s);
    __syncthreads();  // task_s is rewritten for the next task; the tiles are free again
    if (task >= ntask) break;  // uniform
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((cached ? tbs[mid] : tb[mid]) <= task) lo = mid;
      else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const int i_item = __builtin_amdgcn_readfirstlane(perm[lo]);
    const kbe_batch_vjp_item it = uniform_copy(items + i_item);
    const kbe_batch_item &r = it.row;
    int c[VJP_CLASSES];
    vjp_chunks(r, c);
    int local = __builtin_amdgcn_readfirstlane((int)(task - (cached ? tbs[lo] : tb[lo]))), k = 0;
    while (local >= c[k]) local -= c[k++];
    int b0, b1;
    vjp_range(r, k, b0, b1);
    const int vch = vjp_chunk(r.N);
    b0 += local * vch;
    b1 = b0 + vch < b1 ? b0 + vch : b1;
    const int N = r.N, E = N * N, J = r.ntau - 1;
    const int EP = E <= 1 ? 1 : E <= 4 ? 4 : E <= 16 ? 16 : E <= 32 ? 32 : E <= 64 ? 64 : E <= 128 ? 128 : 256;
    const int bps = 256 / EP, sub = tid / EP, e = tid % EP, ei = e / N, ej = e % N;
    const bool valid = e < E;
    // the class's product, cotangent and output array
    const bool ir = r.flags & KBE_OUT_IR, il = r.flags & KBE_OUT_IL;
    const bool itv = (r.flags & KBE_OUT_ITV) && r.ntau > 0;
    int form = F_ZERO;
    const kbe_c128 *Gc = nullptr;
    kbe_c128 *out = nullptr;
    switch (k) {
      case 0: form = ir ? F_GXH : F_ZERO; Gc = it.gIR; out = it.g_sig_ret; break;
      case 1: form = ir ? F_GX : F_ZERO; Gc = it.gIR; out = it.g_sig_ret; break;
      case 2: form = il ? F_GX : F_ZERO; Gc = it.gIL; out = it.g_sig_les; break;
      case 3: form = F_ZERO; out = it.g_sig_les; break;
      case 4: form = ir ? F_XHG : F_ZERO; Gc = it.gIR; out = it.g_col; break;
      case 5: form = ir ? F_GHX : F_ZERO; Gc = it.gIR; out = it.g_row; break;
      case 6: form = il ? F_GHX : F_ZERO; Gc = it.gIL; out = it.g_row; break;
      case 7: form = il ? F_GHX : F_ZERO; Gc = it.gIL; out = it.g_rdiag; break;
      case 8: form = itv ? F_GX : F_ZERO; Gc = it.gItv; out = it.g_sig_tv; break;
      default: form = itv ? F_GHX : F_ZERO; Gc = it.gItv; out = it.g_tv; break;
    }
    // streamed block of output block s, and its scalar
    auto xblk = [&](int s) -> const kbe_c128 * {
      switch (k) {
        case 0: return r.col + (int64_t)s * col_step(r) * E;
        case 1: return r.row + (int64_t)s * E;
        case 2: return s < r.m ? r.row + (int64_t)s * E : r.rdiag;
        case 4: case 5: return r.sig_ret + (int64_t)s * E;
        case 6: return r.sig_les + (int64_t)s * E;
        case 7: return r.sig_les + (int64_t)r.m * E;
        case 8: return r.tv + (int64_t)(J - s) * E;
        default: return r.sig_tv + (int64_t)(J - s) * E;
      }
    };
    auto scal = [&](int s) -> cd {
      switch (k) {
        case 0: case 4: return cd{ldgd(r.wn + s), 0.0};
        case 1: case 5: return cd{-ldgd(r.wn + s), 0.0};
        case 2: case 6: return cd{ldgd(r.wm + s), 0.0};
        case 7: return cd{ldgd(r.wm + r.m), 0.0};
        case 8: return cd{0.0, ldgd(r.wtau + s)};
        default: return cd{0.0, -ldgd(r.wtau + (J - s))};
      }
    };
    if (N == 8) {
      // One v_mfma_f64_4x4x4 product per k-chunk and block: the instruction's four 4x4 blocks
      // b = 2 ti + tj are the four tiles of the 8 x 8 product, so lane l supplies
      // A[4ti + l%4][4kc + l/16] and B[4kc + l/16][4tj + l%4] and holds D[4ti + l/16][4tj + l%4]
      // (ti = (l/8)%2, tj = (l/4)%2).  Operand roles, scaling and the work split as at N = 16
      // below; a wave covers one whole block.
      const int lane = tid & 63, lj = lane & 3, lb = (lane >> 2) & 3, lk = lane >> 4;
      const int ti = lb >> 1, tj = lb & 1;
      const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
      const bool zero = form == F_ZERO;
      const bool xa = form == F_XHG, xt = form == F_GXH, xc = form == F_GXH || form == F_XHG;
      cd gv[2];
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        gv[kc] = czero();
        if (!zero) {
          const int gi = xa ? (4 * kc + lk) * 8 + 4 * tj + lj
                         : (form == F_GHX ? (4 * kc + lk) * 8 + 4 * ti + lj
                                          : (4 * ti + lj) * 8 + 4 * kc + lk);
          gv[kc] = ldg(Gc + gi);
          if (form == F_GHX) gv[kc] = cj(gv[kc]);
        }
      }
      const int xo0 = xa ? lk * 8 + 4 * ti + lj : (xt ? (4 * tj + lj) * 8 + lk : lk * 8 + 4 * tj + lj);
      const int xo1 = xa ? (4 + lk) * 8 + 4 * ti + lj : (xt ? (4 * tj + lj) * 8 + 4 + lk : (4 + lk) * 8 + 4 * tj + lj);
      cd xn[2] = {czero(), czero()}, cn = czero();
      auto fetch8 = [&](int sb) {
        const kbe_c128 *X = xblk(sb);
        xn[0] = ldg(X + xo0);
        xn[1] = ldg(X + xo1);
        cn = scal(sb);
      };
      int s = b0 + wave;
      if (!zero && s < b1) fetch8(s);
      for (; s < b1; s += 4) {
        const cd x0 = xn[0], x1 = xn[1];
        cd cs = cn;
        if (!zero) fetch8(s + 4 < b1 ? s + 4 : b1 - 1);
        if (zero || (k == 6 && s == r.m)) cs = czero();
        double k1 = 0.0, k2 = 0.0, k3 = 0.0;
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
          const cd xv = kc == 0 ? x0 : x1;
          const cd v = cs * (xc ? cj(xv) : xv);
          const cd a = xa ? v : gv[kc], bb = xa ? gv[kc] : v;
          k1 = mfma4b(a.re + a.im, bb.re, k1);
          k2 = mfma4b(a.re, bb.im - bb.re, k2);
          k3 = mfma4b(a.im, bb.re + bb.im, k3);
        }
        stg(out + (int64_t)s * 64 + (4 * ti + lk) * 8 + 4 * tj + lj, cd{k1 - k3, k1 + k2});
      }
      continue;  // the whole workgroup: no barrier inside this branch
    }
    if (N == 16) {
      // One v_mfma_f64_16x16x4 product per block (lane l supplies A[l%16][4kc + l/16] and
      // B[4kc + l/16][l%16] and holds D[l/16 + 4r][l%16]), three real products per complex
      // one as in the small tasks.  The cotangent operand is formed once per task:
      //   G X, G X^dagger: A = G;   G^dagger X: A = G^dagger;   X^dagger G: B = G;
      // the streamed operand is loaded straight into its layout, scaled by the block's scalar:
      //   G X, G^dagger X: B = X;   G X^dagger: B = X^dagger;   X^dagger G: A = X^dagger.
      // Wave w takes the blocks b0 + w, b0 + w + 4, ..., each loaded a block ahead.  No LDS.
      const int lane = tid & 63, lk = lane >> 4, lc = lane & 15;
      const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
      const bool zero = form == F_ZERO;  // nothing is read
      const bool xa = form == F_XHG;     // the streamed operand is A
      const bool xt = form == F_GXH;     // it is read at the transposed position
      const bool xc = form == F_GXH || form == F_XHG;  // and conjugated
      cd gv[4];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        gv[kc] = czero();
        if (!zero) {
          gv[kc] = ldg(Gc + (form == F_GHX || xa ? (4 * kc + lk) * 16 + lc : lc * 16 + 4 * kc + lk));
          if (form == F_GHX) gv[kc] = cj(gv[kc]);
        }
      }
      cd xn[4] = {czero(), czero(), czero(), czero()}, cn = czero();
      auto fetch16 = [&](int sb) {
        const kbe_c128 *X = xblk(sb);
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
          xn[kc] = ldg(X + (xt ? lc * 16 + 4 * kc + lk : (4 * kc + lk) * 16 + lc));
        cn = scal(sb);
      };
      int s = b0 + wave;
      if (!zero && s < b1) fetch16(s);
      for (; s < b1; s += 4) {
        cd x[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) x[kc] = xn[kc];
        cd cs = cn;
        if (!zero) fetch16(s + 4 < b1 ? s + 4 : b1 - 1);
        if (zero || (k == 6 && s == r.m)) cs = czero();  // zero blocks (g_row[m], unselected)
        d4b k1 = {0, 0, 0, 0}, k2 = {0, 0, 0, 0}, k3 = {0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const cd v = cs * (xc ? cj(x[kc]) : x[kc]);
          const cd a = xa ? v : gv[kc], bb = xa ? gv[kc] : v;
          k1 = mfma16b(a.re + a.im, bb.re, k1);
          k2 = mfma16b(a.re, bb.im - bb.re, k2);
          k3 = mfma16b(a.im, bb.re + bb.im, k3);
        }
        kbe_c128 *d = out + (int64_t)s * E;
#pragma unroll
        for (int q = 0; q < 4; ++q) stg(d + (lk + 4 * q) * 16 + lc, cd{k1[q] - k3[q], k1[q] + k2[q]});
      }
      continue;  // the whole workgroup: no barrier inside this branch
    }
    // the cotangent's row ei (G X, G X^dagger), column ej (X^dagger G) or conjugated column ei
    // (G^dagger X) of this thread's element
    cd g[16];
    {
      // loads at clamped, always valid addresses (the output array stands in for an absent
      // cotangent), the unwanted values selected away: no divergent branches
      const kbe_c128 *gp = form == F_ZERO ? out : Gc;
      const int ec = valid ? e : 0, ci = ec / N, cj_ = ec % N;
#pragma unroll
      for (int l = 0; l < 16; ++l) {
        const int lc = l < N ? l : 0;
        const int gi = form == F_XHG ? lc * N + cj_ : form == F_GHX ? lc * N + ci : ci * N + lc;
        cd v = ldg(gp + gi);
        if (form == F_GHX) v = cj(v);  // uniform
        g[l] = (form != F_ZERO && valid && l < N) ? v : czero();
      }
    }
    // steps of VJP_R * bps blocks: thread handles block sub + bps r, r = 0..VJP_R-1, of a step
    const int per = VJP_R * bps;
    const int nstep = (b1 - b0 + per - 1) / per;
    // the step's elements and scalars, loaded a step ahead of their use
    auto fetch = [&](int q, cd (&x)[VJP_R], cd (&sc)[VJP_R]) {
#pragma unroll
      for (int rr = 0; rr < VJP_R; ++rr) {
        const int s = b0 + q * per + rr * bps + sub;
        const bool on = form != F_ZERO && valid && q < nstep && s < b1 && !(k == 6 && s == r.m);
        if (form == F_ZERO) {  // uniform: nothing is read
          x[rr] = sc[rr] = czero();
          continue;
        }
        const int sv = s < b1 ? s : b1 - 1;  // a block of the class: always readable
        const cd xv = ldg(xblk(sv) + (valid ? e : 0));
        const cd cv = scal(sv);
        x[rr] = on ? xv : czero();
        sc[rr] = on ? cv : czero();
      }
    };
    cd xn[VJP_R], cn[VJP_R];
    fetch(0, xn, cn);
    for (int q = 0; q < nstep; ++q) {
      cd xc[VJP_R], cc[VJP_R];
#pragma unroll
      for (int rr = 0; rr < VJP_R; ++rr) {
        xc[rr] = xn[rr];
        cc[rr] = cn[rr];
      }
      fetch(q + 1, xn, cn);
      cd *tile = xs[q & 1];
      // Staging makes every form one loop, acc = sum_l g[l] tile[l N + col]:
      //   G X         : X at (l, j)                    col = j
      //   G^dagger X  : X at (l, j)                    col = j
      //   G X^dagger  : conj(X) transposed, (l, j) <- conj X[j][l]     col = j
      //   X^dagger G  : conj(X) at (l, i)              col = i
      const bool conj_x = form == F_GXH || form == F_XHG;
      const int slot = sub * EP + (form == F_GXH ? ej * N + ei : e);
      if (form != F_ZERO)
#pragma unroll
        for (int rr = 0; rr < VJP_R; ++rr) {
          const cd v = conj_x ? cj(xc[rr]) : xc[rr];
          tile[rr * 256 + (valid ? slot : tid)] = v;
        }
      lds_barrier();
      const int col = form == F_XHG ? ei : ej;
#pragma unroll
      for (int rr = 0; rr < VJP_R; ++rr) {
        const cd *t = tile + rr * 256 + sub * EP + col;
        cd acc = czero();
        if (form != F_ZERO) {
#pragma unroll
          for (int l = 0; l < 16; ++l) {
            if (l < N) {  // uniform
              const cd x = t[l * N];
              acc.re = __builtin_fma(g[l].re, x.re, acc.re);
              acc.re = __builtin_fma(-g[l].im, x.im, acc.re);
              acc.im = __builtin_fma(g[l].re, x.im, acc.im);
              acc.im = __builtin_fma(g[l].im, x.re, acc.im);
            }
          }
        }
        acc = cc[rr] * acc;  // cc is 0 where the block is zero (unselected, or g_row[m])
        const int s = b0 + q * per + rr * bps + sub;
        if (valid && s < b1) stg(out + (int64_t)s * E + e, acc);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------------------
static size_t al256b(size_t x) { return (x + 255) & ~(size_t)255; }

int batch_default_chunk() { return item_chunk(kbe_batch_item{}, 0); }

size_t batch_ws_bytes(const kbe_batch_item *items, int count, int chunk) {
  int64_t parts = 0;
  for (int i = 0; i < count; ++i) {
    int c[4];
    item_chunks(items[i], chunk, c);
    parts += (int64_t)(c[0] + c[1] + c[2] + c[3]) * items[i].N * items[i].N;
  }
  return 2 * al256b(sizeof(int64_t) * (size_t)(count + 1)) + al256b(sizeof(int) * (size_t)count) +
         256 + sizeof(kbe_c128) * (size_t)parts;
}

static int batch_grid() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
  int &c = cached[dev];
  if (c == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_stream, 256, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    c = cus * per_cu;
  }
  return c;
}

hipError_t launch_batch(const kbe_batch_item *items, const kbe_batch_item *items_dev, int count,
                        int chunk, void *ws, hipStream_t st) {
  if (count == 0) return hipSuccess;
  char *w = (char *)ws;
  const size_t tsz = al256b(sizeof(int64_t) * (size_t)(count + 1));
  int64_t *tb = (int64_t *)w;
  int64_t *pb = (int64_t *)(w + tsz);
  int *perm = (int *)(w + 2 * tsz);
  unsigned int *head = (unsigned int *)(w + 2 * tsz + al256b(sizeof(int) * (size_t)count));
  kbe_c128 *parts = (kbe_c128 *)((char *)head + 256);
  int64_t ntask = 0;
  for (int i = 0; i < count; ++i) {
    int c[4];
    item_chunks(items[i], chunk, c);
    ntask += c[0] + c[1] + c[2] + c[3];
  }
  hipLaunchKernelGGL(batch_plan<kbe_batch_item>, dim3(1), dim3(1024), 0, st, items_dev, count, chunk, perm, tb,
                     pb, head);
  if (ntask > 0) {
    int64_t grid = batch_grid();
    const int64_t need = (ntask + 3) / 4;  // four waves per workgroup
    if (grid > need) grid = need;
    hipLaunchKernelGGL(batch_stream, dim3((unsigned)grid), dim3(256), 0, st, items_dev, count,
                       chunk, perm, tb, pb, parts, head);
  }
  hipLaunchKernelGGL(batch_reduce, dim3((unsigned)count), dim3(256), 0, st, items_dev, chunk, pb,
                     parts);
  return hipGetLastError();
}

size_t batch_vjp_ws_bytes(int count) {
  return 2 * al256b(sizeof(int64_t) * (size_t)(count + 1)) + al256b(sizeof(int) * (size_t)count) +
         256;
}

static int batch_vjp_grid() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
  int &c = cached[dev];
  if (c == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_vjp_stream, 256, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    c = cus * per_cu;
  }
  return c;
}

hipError_t launch_batch_vjp(const kbe_batch_vjp_item *items_dev, int count, void *ws,
                            hipStream_t st) {
  if (count == 0) return hipSuccess;
  char *w = (char *)ws;
  const size_t tsz = al256b(sizeof(int64_t) * (size_t)(count + 1));
  int64_t *tb = (int64_t *)w;
  int64_t *pb = (int64_t *)(w + tsz);
  int *perm = (int *)(w + 2 * tsz);
  unsigned int *head = (unsigned int *)(w + 2 * tsz + al256b(sizeof(int) * (size_t)count));
  hipLaunchKernelGGL(batch_plan<kbe_batch_vjp_item>, dim3(1), dim3(1024), 0, st, items_dev, count,
                     0, perm, tb, pb, head);
  hipLaunchKernelGGL(batch_vjp_stream, dim3((unsigned)batch_vjp_grid()), dim3(256), 0, st,
                     items_dev, count, perm, tb, head);
  return hipGetLastError();
}

}  // namespace kbe
