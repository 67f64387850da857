// Quadrature weights on the device (Sec. "Adaptive History Integration",
// Eq. weights and the weight-row recursion of arXiv:2405.08737).
//
// Local weights: the integral over [left, right] of the Lagrange interpolant through k nodes is
// sum_j lam_j g(x_j), where lam solves the moment equations of Eq. weights,
//   sum_j lam_j phi_l(x_j) = int_left^right phi_l(x) dx,   l = 0..k-1,
// solved as in the paper by LU with full pivoting.  The paper writes the equations in the
// monomial basis phi_l = (x - x_0)^l; that Vandermonde matrix has condition ~1e14 at the
// paper's largest order (20), so here the same equations are posed in the Legendre basis
// phi_l = P_l(z), z the affine map of [min(x_0,left), max(x_{k-1},right)] onto [-1, 1]
// (a change of basis: identical solution, condition ~1e6-1e7 at order 20, ~1e2 at order 6).
// k <= KBE_KMAX.
#include "kbe_dev.h"
#include "kbe_internal.h"

namespace kbe {

// One wavefront (a 64-thread workgroup) solves one system: the augmented k x (k+1) matrix lives
// in LDS and every elimination step is spread over the lanes; the pivot is the first element of
// largest modulus in row-major order of the trailing block (the order a serial search uses).
constexpr int KP1 = KBE_KMAX + 1;

struct SolveLds {
  double A[KBE_KMAX][KP1];
  double f[KBE_KMAX];
  double sol[KBE_KMAX];
  int perm[KBE_KMAX];
};

__device__ void wave_solve(const double *x, int k, double left, double right, double *lam,
                           SolveLds &S) {
  const int lane = threadIdx.x;
  if (k == 1) {
    if (lane == 0) lam[0] = right - left;
    return;
  }
  const double lo = fmin(x[0], left), hi = fmax(x[k - 1], right);
  const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
  if (lane < k) {  // column j = lane: P_0..P_{k-1} at node j (three-term recurrence)
    const int j = lane;
    const double z = (x[j] - c) / h;
    double p0 = 1.0, p1 = z;
    S.A[0][j] = 1.0;
    S.A[1][j] = z;
    for (int l = 1; l + 1 < k; ++l) {
      const double p2 = ((2 * l + 1) * z * p1 - l * p0) / (l + 1);
      p0 = p1;
      p1 = p2;
      S.A[l + 1][j] = p2;
    }
    S.perm[j] = j;
  }
  if (lane == 63) {  // right-hand side: h * int_{za}^{zb} P_l, int P_l = (P_{l+1} - P_{l-1})/(2l+1)
    const double za = (left - c) / h, zb = (right - c) / h;
    double a0 = 1.0, a1 = za, b0 = 1.0, b1 = zb;
    S.A[0][k] = h * (zb - za);
    for (int l = 1; l < k; ++l) {
      const double a2 = ((2 * l + 1) * za * a1 - l * a0) / (l + 1);
      const double b2 = ((2 * l + 1) * zb * b1 - l * b0) / (l + 1);
      S.A[l][k] = h * ((b2 - b0) - (a2 - a0)) / (2 * l + 1);
      a0 = a1;
      a1 = a2;
      b0 = b1;
      b1 = b2;
    }
  }
  __syncthreads();
  for (int s = 0; s < k; ++s) {
    const int w = k - s;
    double best = -1.0;
    int bi = 1 << 30;
    for (int e = lane; e < w * w; e += 64) {  // increasing e: first maximum of this lane
      const double v = fabs(S.A[s + e / w][s + e % w]);
      if (v > best) {
        best = v;
        bi = e;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {  // maximum, ties to the smaller index
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const int pr = s + bi / w, pc = s + bi % w;
    if (pr != s)
      for (int cc = lane; cc <= k; cc += 64) {
        const double tmp = S.A[s][cc];
        S.A[s][cc] = S.A[pr][cc];
        S.A[pr][cc] = tmp;
      }
    __syncthreads();
    if (pc != s) {
      for (int r = lane; r < k; r += 64) {
        const double tmp = S.A[r][s];
        S.A[r][s] = S.A[r][pc];
        S.A[r][pc] = tmp;
      }
      if (lane == 0) {
        const int tp = S.perm[s];
        S.perm[s] = S.perm[pc];
        S.perm[pc] = tp;
      }
    }
    __syncthreads();
    for (int r = s + 1 + lane; r < k; r += 64) S.f[r] = S.A[r][s] / S.A[s][s];
    __syncthreads();
    const int wc = k - s + 1;
    for (int e = lane; e < (w - 1) * wc; e += 64) {
      const int r = s + 1 + e / wc, cc = s + e % wc;
      S.A[r][cc] -= S.f[r] * S.A[s][cc];
    }
    __syncthreads();
  }
  if (lane == 0) {
    for (int s = k - 1; s >= 0; --s) {
      double acc = S.A[s][k];
      for (int cc = s + 1; cc < k; ++cc) acc -= S.A[s][cc] * S.sol[cc];
      S.sol[s] = acc / S.A[s][s];
    }
    for (int s = 0; s < k; ++s) lam[S.perm[s]] = S.sol[s];
  }
}

// lam[p][0..k_p), k_p = min(order[p], p+1), nodes t[p-k_p+1 .. p], interval [t_{p-1}, t_p].
// One 64-thread workgroup per interval.
__global__ void __launch_bounds__(64) local_weights_kernel(const double *t, const int32_t *order,
                                                           int nt, double *lam, int32_t *kk) {
  __shared__ SolveLds S;
  __shared__ double l[KBE_KMAX];
  const int p = blockIdx.x + 1;
  if (p >= nt) return;
  int k = order[p] < 1 ? 1 : (order[p] > KBE_KMAX ? KBE_KMAX : order[p]);  // in range when valid
  k = k < p + 1 ? k : p + 1;
  if (threadIdx.x == 0) kk[p] = k;
  wave_solve(t + (p - k + 1), k, t[p - 1], t[p], l, S);
  __syncthreads();
  if (threadIdx.x < KBE_KMAX) lam[(int64_t)p * KBE_KMAX + threadIdx.x] = (int)threadIdx.x < k ? l[threadIdx.x] : 0.0;
}

// Composite rows: w[n][s] = sum over intervals p <= n whose nodes include s of the
// local weight of s, summed in increasing p (the order of the row recursion).
__global__ void __launch_bounds__(256) composite_kernel(const double *lam, const int32_t *kk,
                                                        int nt, double *w) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nt * nt) return;
  int n = (int)(idx / nt), s = (int)(idx % nt);
  double acc = 0.0;
  if (s <= n) {
    int p0 = s > 1 ? s : 1;
    int p1 = n < s + KBE_KMAX - 1 ? n : s + KBE_KMAX - 1;
    for (int p = p0; p <= p1; ++p) {
      int a = p - kk[p] + 1;
      if (a <= s) acc += lam[(int64_t)p * KBE_KMAX + (s - a)];
    }
  }
  w[idx] = acc;
}

// Unit-spacing table for the uniform tau grid: tab[kk-1][r][i], the weight of node i
// (of nodes 0..kk-1) for the interval [r-1, r], r = 0..kk-1 (r = 0 occurs for kk = 1 only:
// the single-node rule on the interval that ends at its node).  One wave per (kk, r).
__global__ void __launch_bounds__(64) tau_table_kernel(double *tab, int K) {
  __shared__ SolveLds S;
  __shared__ double l[KBE_KMAX];
  __shared__ double x[KBE_KMAX];
  const int id = blockIdx.x;
  const int kk = id / KBE_KMAX + 1, r = id % KBE_KMAX;
  double *out = tab + ((int64_t)(kk - 1) * KBE_KMAX + r) * KBE_KMAX;
  if (threadIdx.x < KBE_KMAX) out[threadIdx.x] = 0.0;
  if (kk > K || r >= kk || (r == 0 && kk > 1)) return;  // uniform per workgroup
  if (threadIdx.x < KBE_KMAX) x[threadIdx.x] = (double)threadIdx.x;
  __syncthreads();
  wave_solve(x, kk, r - 1.0, (double)r, l, S);
  __syncthreads();
  if ((int)threadIdx.x < kk) out[threadIdx.x] = l[threadIdx.x];
}

// wf[j][l]: integral over [0, tau_j]; interval p in [1, j] uses kk = min(K, j+1) nodes on the
// window starting at a = clamp(p-kk+1, 0, j-kk+1).
__global__ void __launch_bounds__(256) tau_fwd_kernel(const double *tab, int ntau, int K,
                                                      double h, double *wf) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ntau * ntau) return;
  int j = (int)(idx / ntau), l = (int)(idx % ntau);
  double acc = 0.0;
  if (l <= j && j > 0) {
    int kk = K < j + 1 ? K : j + 1;
    for (int p = 1; p <= j; ++p) {
      int a = p - kk + 1;
      if (a < 0) a = 0;
      if (a > j - kk + 1) a = j - kk + 1;
      if (l >= a && l < a + kk) acc += h * tab[((int64_t)(kk - 1) * KBE_KMAX + (p - a)) * KBE_KMAX + (l - a)];
    }
  }
  wf[idx] = acc;
}

__global__ void tau_full_kernel(const double *wf, int ntau, double *wtau) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= ntau) return;
  int J = ntau - 1;
  wtau[l] = 0.5 * (wf[(int64_t)J * ntau + l] + wf[(int64_t)J * ntau + (J - l)]);
}

// Local weights of interval p for every node count k = 1..min(order[p], p+1) (the time-stepping
// rules of elements whose history starts inside the interval's window): lam[p][k-1][i] for the
// nodes t[p-k+1+i]; zero elsewhere.  One 64-thread workgroup per (p, k).
__global__ void __launch_bounds__(64) step_weights_kernel(const double *t, const int32_t *order,
                                                          int nt, double *lam) {
  __shared__ SolveLds S;
  __shared__ double l[KBE_KMAX];
  const int p = blockIdx.x / KBE_KMAX, k = blockIdx.x % KBE_KMAX + 1;
  double *out = lam + ((int64_t)p * KBE_KMAX + (k - 1)) * KBE_KMAX;
  if (threadIdx.x < KBE_KMAX) out[threadIdx.x] = 0.0;
  if (p < 1 || p >= nt) return;  // uniform per workgroup
  int kp = order[p] < 1 ? 1 : (order[p] > KBE_KMAX ? KBE_KMAX : order[p]);
  kp = kp < p + 1 ? kp : p + 1;
  if (k > kp) return;
  wave_solve(t + (p - k + 1), k, t[p - 1], t[p], l, S);
  __syncthreads();
  if ((int)threadIdx.x < k) out[threadIdx.x] = l[threadIdx.x];
}

// Rules of one interval n = [t_{n-1}, t_n] for an adaptive step, t_n = tn (also stored in t[n] by
// workgroup 0; every workgroup takes node n from the argument): am[k-1][i], the local weights
// of Eq. weights on the k nodes t_{n-k+1..n} (k = 1..min(kam, n+1)), and ab[q-1][i], the integral
// over the same interval of the Lagrange basis on the q nodes t_{n-q..n-1} (the predictor,
// q = 1..min(kab, n)); other entries zero.  Each weight is the integral of its Lagrange basis
// polynomial (degree < KBE_KMAX) by a Gauss-Legendre rule with GL_M points, exact for degree
// < 2 GL_M: the same numbers as the moment equations, without their conditioning at high order.
// One 64-thread workgroup per (table, k), one thread per weight.
constexpr int GL_M = 12;
struct GLRule {
  double x[GL_M], w[GL_M];  // nodes and weights on [-1, 1]
};
static_assert(2 * GL_M > KBE_KMAX - 1, "the rule must integrate degree KBE_KMAX - 1 exactly");

__global__ void __launch_bounds__(64) interval_weights_kernel(double *t, int n, double tn, int kam,
                                                              int kab, double *am, double *ab,
                                                              GLRule g) {
  const int tab = blockIdx.x / KBE_KMAX, k = blockIdx.x % KBE_KMAX + 1;
  double *out = (tab == 0 ? am : ab) + (int64_t)(k - 1) * KBE_KMAX;
  const int j = threadIdx.x;
  __shared__ double x[KBE_KMAX];
  const int kmx = tab == 0 ? (kam < n + 1 ? kam : n + 1) : (kab < n ? kab : n);
  const bool live = n >= 1 && k <= kmx;                 // uniform per workgroup
  const int first = tab == 0 ? n - k + 1 : n - k;      // nodes t[first .. first + k - 1]
  if (live && j < k) x[j] = first + j == n ? tn : t[first + j];
  __syncthreads();
  if (blockIdx.x == 0 && j == 0) t[n] = tn;  // no workgroup reads t[n]: node n is tn
  if (j >= KBE_KMAX) return;
  if (!live || j >= k) {
    out[j] = 0.0;
    return;
  }
  const double a = t[n - 1], b = tn, half = 0.5 * (b - a), mid = 0.5 * (a + b);
  double den = 1.0;
  for (int i = 0; i < k; ++i)
    if (i != j) den *= x[j] - x[i];
  double acc = 0.0;
  for (int m = 0; m < GL_M; ++m) {
    const double s = mid + half * g.x[m];
    double pr = 1.0;
    for (int i = 0; i < k; ++i)
      if (i != j) pr *= s - x[i];
    acc += g.w[m] * pr;
  }
  out[j] = half * acc / den;
}

// The GL_M-point Gauss-Legendre rule on [-1, 1]: Newton's method on the three-term recurrence of
// the Legendre polynomials from the usual cosine guesses.
static GLRule gauss_legendre() {
  GLRule g{};
  const int m = GL_M;
  for (int i = 0; i < m; ++i) {
    double z = cos(M_PI * (i + 0.75) / (m + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int l = 1; l < m; ++l) {
        const double p2 = ((2.0 * l + 1.0) * z * p1 - l * p0) / (l + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = m * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    g.x[i] = z;
    g.w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  return g;
}

// Grid check on the device: status = 0, or KBE_EINVAL (t[0] != 0 or t not increasing), or
// KBE_ERANGE (an order outside 1..KBE_KMAX).  One workgroup; a fixed-order reduction.
__global__ void __launch_bounds__(256) grid_check_kernel(const double *t, const int32_t *order,
                                                         int nt, int32_t *status) {
  __shared__ int bad_t, bad_o;
  if (threadIdx.x == 0) {
    bad_t = t[0] != 0.0;
    bad_o = 0;
  }
  __syncthreads();
  for (int p = 1 + threadIdx.x; p < nt; p += blockDim.x) {
    if (!(t[p] > t[p - 1])) atomicOr(&bad_t, 1);
    if (order[p] < 1 || order[p] > KBE_KMAX) atomicOr(&bad_o, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) status[0] = bad_t ? (int32_t)KBE_EINVAL : (bad_o ? (int32_t)KBE_ERANGE : 0);
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t weights_ws_bytes(int nt, int ntau) {
  size_t b = 0;
  b += align256(sizeof(double) * nt);                    // t
  b += align256(sizeof(int32_t) * nt);                   // order
  b += align256(sizeof(double) * (size_t)nt * KBE_KMAX); // lam
  b += align256(sizeof(int32_t) * nt);                   // kk
  if (ntau > 0) b += align256(sizeof(double) * KBE_KMAX * KBE_KMAX * KBE_KMAX);
  return b;
}

// Weights from a grid already in device memory (t_d, o_d); ws holds the rest of the layout of
// weights_ws_bytes (its first two slots, for a host copy of the grid, stay unused).
hipError_t launch_weights_dev(const double *t_d, const int32_t *o_d, int nt, int ntau,
                              double beta, int tau_order, double *w, double *wtau, double *wf,
                              void *ws, hipStream_t st) {
  char *base = (char *)ws;
  base += align256(sizeof(double) * nt);
  base += align256(sizeof(int32_t) * nt);
  double *lam = (double *)base;
  base += align256(sizeof(double) * (size_t)nt * KBE_KMAX);
  int32_t *kk = (int32_t *)base;
  base += align256(sizeof(int32_t) * nt);
  double *tab = (double *)base;
  if (nt > 1)
    hipLaunchKernelGGL(local_weights_kernel, dim3(nt - 1), dim3(64), 0, st, t_d, o_d, nt, lam, kk);
  int64_t tot = (int64_t)nt * nt;
  hipLaunchKernelGGL(composite_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, lam,
                     kk, nt, w);
  if (ntau > 0) {
    hipLaunchKernelGGL(tau_table_kernel, dim3(KBE_KMAX * KBE_KMAX), dim3(64), 0, st, tab,
                       tau_order);
    int64_t tt = (int64_t)ntau * ntau;
    hipLaunchKernelGGL(tau_fwd_kernel, dim3((unsigned)((tt + 255) / 256)), dim3(256), 0, st, tab,
                       ntau, tau_order, beta / (ntau - 1), wf);
    hipLaunchKernelGGL(tau_full_kernel, dim3((ntau + 255) / 256), dim3(256), 0, st, wf, ntau,
                       wtau);
  }
  return hipGetLastError();
}

hipError_t launch_weights(const kbe_grid *g, double *w, double *wtau, double *wf, void *ws,
                          hipStream_t st) {
  const int nt = g->nt;
  double *t_d = (double *)ws;
  int32_t *o_d = (int32_t *)((char *)ws + align256(sizeof(double) * nt));
  hipError_t e = hipMemcpyAsync(t_d, g->t, sizeof(double) * nt, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(o_d, g->order, sizeof(int32_t) * nt, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return launch_weights_dev(t_d, o_d, nt, g->ntau, g->beta, g->tau_order, w, wtau, wf, ws, st);
}

hipError_t launch_grid_check(const double *t, const int32_t *order, int nt, int32_t *status,
                             hipStream_t st) {
  hipLaunchKernelGGL(grid_check_kernel, dim3(1), dim3(256), 0, st, t, order, nt, status);
  return hipGetLastError();
}

hipError_t launch_interval_weights(double *t, int n, double tn, int kam, int kab, double *am,
                                   double *ab, hipStream_t st) {
  static const GLRule g = gauss_legendre();
  hipLaunchKernelGGL(interval_weights_kernel, dim3(2 * KBE_KMAX), dim3(64), 0, st, t, n, tn, kam,
                     kab, am, ab, g);
  return hipGetLastError();
}

hipError_t launch_step_weights(const double *t, const int32_t *order, int nt, double *lam,
                               hipStream_t st) {
  hipLaunchKernelGGL(step_weights_kernel, dim3((unsigned)nt * KBE_KMAX), dim3(64), 0, st, t, order,
                     nt, lam);
  return hipGetLastError();
}

}  // namespace kbe
