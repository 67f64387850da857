// Second-Born (GF2) self-energy row with a general four-index interaction (Eq. SE of
// arXiv:2405.08737):
//   Sigma_ij = sum_{f,d,e,a,b,c} U_ifde Uex_jabc A_fb A_ea C_cd,   Uex_jabc = 2 U_jbac - U_jabc,
// with (A, C) = (G^<(t_n,t_s), G^>(t_s,t_n)) for Sigma^<, (G^>(t_n,t_s), G^<(t_s,t_n)) for
// Sigma^>, and (G^](t_n,tau_l), G^[(tau_l,t_n)) for Sigma^].  U is real, U[i][f][d][e] = U_ifde.
//
// The six-fold sum factors into four contractions of N^5 multiply-adds each.  For one output
// column j:
//   S1_a[b][d] = sum_c Uex[j][a][b][c] C[c][d]      (for each a: an N x N block)
//   S2[f][a][d] = sum_b A[f][b] S1_a[b][d]           (N^3, kept in LDS)
//   S3_f[e][d] = sum_a A[e][a] S2[f][a][d]           (for each f: an N x N block)
//   Sigma_ij   = sum_f sum_d sum_e U[i][f][d][e] S3_f[e][d]
// One workgroup per time pair (both Sigma^< and Sigma^> for a real-time pair, so it writes
// Sigma^R = Sigma^> - Sigma^< itself), blocks padded with zeros to NP = 4, 8 or 16 (exact: the
// padding adds exact zeros).  N <= 8 runs on the vector ALU with NP x NP threads, as follows;
// 9 <= N <= 16 runs on the matrix cores (gf2_mfma16_kernel, below).  Thread (x, y) keeps row x
// of A and column y of C
// in registers; S1_a and S3_f pass through double-buffered LDS tiles, S2 through one NP^3 tile;
// thread (i, p) sums the part d = p of column j's last contraction and the NP threads of a row
// add their parts with lane shuffles.  U and Uex are read from a zero-padded copy in the
// workspace (L2-resident: 2 NP^4 doubles).
#include "kbe_dev.h"
#include "kbe_internal.h"

namespace kbe {

namespace {

struct Gf2Args {
  int N, ntau, J, n;
  int64_t ldt;
  const kbe_c128 *kp, *rdiag, *tv;
  const double *U, *X;  // padded U and Uex, [NP]^4
  kbe_c128 *ret, *les, *stv;
};

__device__ __forceinline__ void cfma(cd &acc, cd a, cd b) {
  acc.re = __builtin_fma(a.re, b.re, acc.re);
  acc.re = __builtin_fma(-a.im, b.im, acc.re);
  acc.im = __builtin_fma(a.re, b.im, acc.im);
  acc.im = __builtin_fma(a.im, b.re, acc.im);
}
__device__ __forceinline__ void rfma(cd &acc, double u, cd b) {
  acc.re = __builtin_fma(u, b.re, acc.re);
  acc.im = __builtin_fma(u, b.im, acc.im);
}

// Elements of the blocks a real-time pair (n, s), s <= n, reads through the storage symmetries:
// G^<(n,s) = -kp[s][n]^dagger (s < n), G^R(n,s) = kp[n][s] (s < n) or rdiag[n] (s = n),
// G^>(n,s) = G^R(n,s) + G^<(n,s), G^<(s,n) = kp[s][n], G^>(s,n) = -G^>(n,s)^dagger (s < n).
struct PairBlocks {
  const kbe_c128 *up, *lo, *rd;  // kp[s][n], kp[n][s], rdiag[n]
  int N;
  bool diag;
  __device__ cd les_ns(int x, int y) const {
    return diag ? ld(up + x * N + y) : -cj(ld(up + y * N + x));
  }
  __device__ cd gtr_ns(int x, int y) const {
    return (diag ? ld(rd + x * N + y) : ld(lo + x * N + y)) + les_ns(x, y);
  }
  __device__ cd les_sn(int x, int y) const { return ld(up + x * N + y); }
  __device__ cd gtr_sn(int x, int y) const {
    return diag ? gtr_ns(x, y) : -cj(gtr_ns(y, x));
  }
};

// Sigma block of one (A, C) pair; thread (x, y) supplies A[x][.] and C[.][y] and gets back
// Sigma[x][y].  Every thread of the workgroup calls it.
template <int NP>
__device__ cd gf2_block(const Gf2Args &g, const cd (&Ar)[NP], const cd (&Cc)[NP], cd *S2,
                        cd (*S1)[NP * NP], cd (*S3)[NP * NP], int x, int y) {
  cd out = czero();
  for (int j = 0; j < NP; ++j) {
    // S2[f][a][d] for every a (thread: b = x then f = x, d = y)
    for (int a = 0; a < NP; ++a) {
      const double *xr = g.X + (((int64_t)j * NP + a) * NP + x) * NP;  // Uex[j][a][x][.]
      cd s1 = czero();
#pragma unroll
      for (int c = 0; c < NP; ++c) rfma(s1, xr[c], Cc[c]);
      cd *t1 = S1[a & 1];
      t1[x * NP + y] = s1;
      lds_barrier();
      cd s2 = czero();
#pragma unroll
      for (int b = 0; b < NP; ++b) cfma(s2, Ar[b], t1[b * NP + y]);
      S2[(x * NP + a) * NP + y] = s2;
    }
    lds_barrier();
    // column j of Sigma (thread: e = x then i = x, d = p = y)
    cd part = czero();
    for (int f = 0; f < NP; ++f) {
      cd s3 = czero();
#pragma unroll
      for (int a = 0; a < NP; ++a) cfma(s3, Ar[a], S2[(f * NP + a) * NP + y]);
      cd *t3 = S3[f & 1];
      t3[x * NP + y] = s3;
      lds_barrier();
      const double *ur = g.U + (((int64_t)x * NP + f) * NP + y) * NP;  // U[x][f][y][.]
#pragma unroll
      for (int e = 0; e < NP; ++e) rfma(part, ur[e], t3[e * NP + y]);
    }
    // sum over p = y within the row's NP lanes
#pragma unroll
    for (int off = 1; off < NP; off <<= 1) {
      part.re += __shfl_xor(part.re, off, NP);
      part.im += __shfl_xor(part.im, off, NP);
    }
    if (y == j) out = part;
    lds_barrier();  // S2 and the tiles are rewritten for the next column
  }
  return out;
}

template <int NP>
__global__ void __launch_bounds__(NP * NP) gf2_row_kernel(Gf2Args g) {
  __shared__ cd S2[NP * NP * NP];
  __shared__ cd S1[2][NP * NP];
  __shared__ cd S3[2][NP * NP];
  const int tid = threadIdx.x, x = tid / NP, y = tid % NP, N = g.N;
  const int job = blockIdx.x;
  const int64_t E = (int64_t)N * N;
  cd Ar[NP], Cc[NP];
  if (job <= g.n) {  // real-time pair (n, s = job): Sigma^< then Sigma^>
    const int s = job;
    PairBlocks P{g.kp + ((int64_t)s * g.ldt + g.n) * E, g.kp + ((int64_t)g.n * g.ldt + s) * E,
                 g.rdiag + (int64_t)g.n * E, N, s == g.n};
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      Ar[k] = (x < N && k < N) ? P.les_ns(x, k) : czero();
      Cc[k] = (k < N && y < N) ? P.gtr_sn(k, y) : czero();
    }
    const cd sl = gf2_block<NP>(g, Ar, Cc, S2, S1, S3, x, y);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      Ar[k] = (x < N && k < N) ? P.gtr_ns(x, k) : czero();
      Cc[k] = (k < N && y < N) ? P.les_sn(k, y) : czero();
    }
    const cd sg = gf2_block<NP>(g, Ar, Cc, S2, S1, S3, x, y);
    if (x < N && y < N) {
      st(g.les + s * E + x * N + y, sl);
      st(g.ret + s * E + x * N + y, sg - sl);
    }
  } else {  // mixed branch: A = G^](t_n, tau_l), C = G^[(tau_l, t_n) = G^](t_n, tau_{J-l})^dagger
    const int l = job - g.n - 1;
    const kbe_c128 *a = g.tv + ((int64_t)g.n * g.ntau + l) * E;
    const kbe_c128 *c = g.tv + ((int64_t)g.n * g.ntau + (g.J - l)) * E;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      Ar[k] = (x < N && k < N) ? ld(a + x * N + k) : czero();
      Cc[k] = (k < N && y < N) ? cj(ld(c + y * N + k)) : czero();
    }
    const cd sm = gf2_block<NP>(g, Ar, Cc, S2, S1, S3, x, y);
    if (x < N && y < N) st(g.stv + (int64_t)l * E + x * N + y, sm);
  }
}

// ---------------------------------------------------------------------------------------------
// 9 <= N <= 16: the three contractions of each column that involve A or C run on the FP64 matrix
// cores as 16 x 16 x 16 products (v_mfma_f64_16x16x4: lane l supplies A[l%16][k] and B[k][l%16]
// for k = 4 kc + l/16 and receives D[l/16 + 4 r][l%16], r = 0..3).  The left operand is supplied
// with its rows permuted, row p(i) = 4 (i % 4) + i / 4 in slot i, so that lane l receives rows
// 4 (l/16) + r of the product: four consecutive rows per lane.  Complex products take three
// real ones, k1 = (ar + ai) br, k2 = ar (bi - br), k3 = ai (br + bi), Re = k1 - k3, Im = k1 + k2.
// A stays in registers as the left operand of S2 and S3 for the whole call, C as the right
// operand of S1.  Per column j:
//   phase 1, wave w, a = w, w + 4, ...:  S1_a = Uex[j][a] C (two real products) goes through
//     S2's a-slice (owned by the wave in this phase) into the operand layout, then
//     S2[.][a][.] = A S1_a overwrites that slice;
//   phase 2, wave w, f = w, w + 4, ...:  S3_f = A S2[f] (operands read straight from S2), then
//     each lane adds its four S3_f entries times U[i][f][d][e] into sixteen partial sums (one per
//     i), reduced over the wave by a reduce-scatter butterfly and over the four waves in order;
//     wave 0 writes column j (Sigma^R = Sigma^> - Sigma^< from the Sigma^< value it wrote).
// ---------------------------------------------------------------------------------------------
typedef double __attribute__((ext_vector_type(4))) d4;

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

struct AOp {  // left operand A[l%16][4 kc + l/16], kc = 0..3, with ar + ai for the first product
  double r[4], i[4], s[4];
};

// Gauss products of A (registers) with a right operand whose kc-th element this lane reads at
// B[kc]; returns the lane's four D entries as (re, im).
template <typename LoadB>
__device__ __forceinline__ void cgemm16(const AOp &A, LoadB loadB, d4 &re, d4 &im) {
  d4 k1 = {0, 0, 0, 0}, k2 = {0, 0, 0, 0}, k3 = {0, 0, 0, 0};
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const cd b = loadB(kc);
    k1 = mfma16(A.s[kc], b.re, k1);
    k2 = mfma16(A.r[kc], b.im - b.re, k2);
    k3 = mfma16(A.i[kc], b.re + b.im, k3);
  }
  re = k1 - k3;
  im = k1 + k2;
}

__global__ void __launch_bounds__(256) gf2_mfma16_kernel(Gf2Args g) {
  constexpr int NP = 16;
  __shared__ cd S2[NP * NP * NP];   // [f][a][d]
  __shared__ cd R[4][NP];           // per-wave column sums
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lq = lane >> 4;
  const int pr = 4 * (li & 3) + (li >> 2);  // left-operand row this lane supplies
  const int N = g.N, job = blockIdx.x;
  const int64_t E = (int64_t)N * N;
  const bool realtime = job <= g.n;
  const int s = job, l = job - g.n - 1;
  PairBlocks P{g.kp + ((int64_t)s * g.ldt + g.n) * E, g.kp + ((int64_t)g.n * g.ldt + s) * E,
               g.rdiag + (int64_t)g.n * E, N, s == g.n};
  const kbe_c128 *ta = g.tv + ((int64_t)g.n * g.ntau + (realtime ? 0 : l)) * E;
  const kbe_c128 *tc = g.tv + ((int64_t)g.n * g.ntau + (realtime ? 0 : g.J - l)) * E;
  const int ncomp = realtime ? 2 : 1;
  for (int comp = 0; comp < ncomp; ++comp) {
    AOp A;
    double cr[4], ci[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int k = 4 * kc + lq;
      cd a = czero(), c = czero();
      if (pr < N && k < N) a = !realtime ? ld(ta + pr * N + k)
                               : comp == 0 ? P.les_ns(pr, k) : P.gtr_ns(pr, k);
      if (li < N && k < N) c = !realtime ? cj(ld(tc + li * N + k))  // conj(tv[J-l][li][k])
                               : comp == 0 ? P.gtr_sn(k, li) : P.les_sn(k, li);
      A.r[kc] = a.re;
      A.i[kc] = a.im;
      A.s[kc] = a.re + a.im;
      cr[kc] = c.re;
      ci[kc] = c.im;
    }
    for (int j = 0; j < NP; ++j) {
      for (int a = w; a < NP; a += 4) {
        const double *xr = g.X + (((int64_t)j * NP + a) * NP + pr) * NP + lq;  // Uex[j][a][pr][.]
        d4 s1r = {0, 0, 0, 0}, s1i = {0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const double x = xr[4 * kc];
          s1r = mfma16(x, cr[kc], s1r);
          s1i = mfma16(x, ci[kc], s1i);
        }
        cd *t = S2 + a * NP;  // the a-slice: element (row, d) at t[row * NP * NP + d]
#pragma unroll
        for (int r = 0; r < 4; ++r) t[(4 * lq + r) * NP * NP + li] = cd{s1r[r], s1i[r]};
        wave_lds_sync();
        d4 re, im;
        cgemm16(A, [&](int kc) { return t[(4 * kc + lq) * NP * NP + li]; }, re, im);
        wave_lds_sync();  // every lane has read S1_a before the slice is overwritten
#pragma unroll
        for (int r = 0; r < 4; ++r) t[(4 * lq + r) * NP * NP + li] = cd{re[r], im[r]};
      }
      lds_barrier();
      cd acc[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) acc[i] = czero();
      for (int f = w; f < NP; f += 4) {
        d4 re, im;
        cgemm16(A, [&](int kc) { return S2[(f * NP + 4 * kc + lq) * NP + li]; }, re, im);
        // this lane's S3_f entries: e = 4 lq + r, d = li
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const d4 u = *(const d4 *)(g.U + (((int64_t)i * NP + f) * NP + li) * NP + 4 * lq);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc[i].re = __builtin_fma(u[r], re[r], acc[i].re);
            acc[i].im = __builtin_fma(u[r], im[r], acc[i].im);
          }
        }
      }
      // reduce-scatter over the wave: after the steps on lane bits 5..2 lane l holds the part of
      // i = 8 b5 + 4 b4 + 2 b3 + b2; bits 1 and 0 are summed last
#pragma unroll
      for (int step = 0; step < 4; ++step) {
        const int m = 32 >> step, c = 8 >> step;
        const bool up = lane & m;
#pragma unroll
        for (int k = 0; k < c; ++k) {
          const cd lo = acc[k], hi = acc[k + c];
          const cd send = up ? lo : hi, keep = up ? hi : lo;
          acc[k].re = keep.re + __shfl_xor(send.re, m);
          acc[k].im = keep.im + __shfl_xor(send.im, m);
        }
      }
      acc[0].re += __shfl_xor(acc[0].re, 2);
      acc[0].im += __shfl_xor(acc[0].im, 2);
      acc[0].re += __shfl_xor(acc[0].re, 1);
      acc[0].im += __shfl_xor(acc[0].im, 1);
      if ((lane & 3) == 0) {
        const int i = 8 * ((lane >> 5) & 1) + 4 * ((lane >> 4) & 1) + 2 * ((lane >> 3) & 1) +
                      ((lane >> 2) & 1);
        R[w][i] = acc[0];
      }
      lds_barrier();
      if (w == 0 && lane < N && j < N) {
        const cd v = ((R[0][lane] + R[1][lane]) + R[2][lane]) + R[3][lane];
        const int64_t o = lane * N + j;
        if (!realtime) st(g.stv + (int64_t)l * E + o, v);
        else if (comp == 0) st(g.les + s * E + o, v);
        else st(g.ret + s * E + o, v - ld(g.les + s * E + o));  // written by this lane above
      }
    }
  }
}

// Zero-padded U and Uex_jabc = 2 U_jbac - U_jabc, [NP]^4 each.
__global__ void __launch_bounds__(256) gf2_prep_kernel(const double *U, int N, int NP, double *Up,
                                                       double *Xp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)NP * NP * NP * NP;
  if (t >= tot) return;
  const int q3 = (int)(t % NP), q2 = (int)(t / NP % NP), q1 = (int)(t / NP / NP % NP),
            q0 = (int)(t / NP / NP / NP);
  const bool in = q0 < N && q1 < N && q2 < N && q3 < N;
  auto at = [&](int a, int b, int c, int d) { return U[(((int64_t)a * N + b) * N + c) * N + d]; };
  Up[t] = in ? at(q0, q1, q2, q3) : 0.0;
  Xp[t] = in ? 2.0 * at(q0, q2, q1, q3) - at(q0, q1, q2, q3) : 0.0;
}

int gf2_np(int N) { return N <= 4 ? 4 : N <= 8 ? 8 : 16; }

}  // namespace

size_t gf2_ws_bytes(int N) {
  const size_t np = (size_t)gf2_np(N);
  return 2 * np * np * np * np * sizeof(double);
}

hipError_t launch_sigma_gf2(const kbe_green *G, const double *U, int n, const kbe_sigma_row *out,
                            void *ws, hipStream_t st) {
  const int NP = gf2_np(G->N);
  const int64_t np4 = (int64_t)NP * NP * NP * NP;
  double *Up = (double *)ws, *Xp = Up + np4;
  hipLaunchKernelGGL(gf2_prep_kernel, dim3((unsigned)((np4 + 255) / 256)), dim3(256), 0, st, U,
                     G->N, NP, Up, Xp);
  Gf2Args g{G->N, G->ntau, G->ntau - 1, n, G->ldt, G->kp, G->rdiag, G->tv, Up, Xp,
            out->ret, out->les, out->tv};
  const unsigned jobs = (unsigned)(n + 1 + G->ntau);
  switch (NP) {
    case 4: hipLaunchKernelGGL(gf2_row_kernel<4>, dim3(jobs), dim3(16), 0, st, g); break;
    case 8: hipLaunchKernelGGL(gf2_row_kernel<8>, dim3(jobs), dim3(64), 0, st, g); break;
    default: hipLaunchKernelGGL(gf2_mfma16_kernel, dim3(jobs), dim3(256), 0, st, g); break;
  }
  return hipGetLastError();
}

}  // namespace kbe
