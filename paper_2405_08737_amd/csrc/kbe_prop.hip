// Fixed-grid propagation of the Kadanoff-Baym equations and its adjoint, on gfx950.
//
// arXiv:2405.08737 propagates G^< above the t = t' diagonal (Eq. KBE1) and G^> below it
// (Eq. KBE2), with G^] (Eq. KBE3), stacked as one state vector in a single time variable: the
// values of the newest row and column.  Here the grid and the orders are fixed, and the
// unknowns are the library's KP storage (kp[m][n] = G^<(t_m,t_n) for m <= n, kp[n][m] =
// G^R(t_n,t_m) = G^> - G^< for m < n, rdiag = G^R(t,t) = -i, tv[n][j] = G^](t_n,tau_j)).  The
// state of step n consists of these elements, each an N x N block obeying an ODE in t~ = t_n:
//   U_m  kp[m][n]  f = i (kp[m][n] eps - C^<(n,m)^dagger)                  (Eq. KBE1 at (t_m,t~))
//   R_m  kp[n][m]  f = -i (eps kp[n][m] + C^>(n,m) - C^<(n,m))             (Eq. KBE2, G^> - G^<)
//   D    kp[n][n]  f = -i [eps, kp[n][n]] - i (C^<(n,n) + C^<(n,n)^dagger) (both derivatives)
//   T_j  tv[n][j]  f = -i (eps tv[n][j] + J^](n,j))                        (Eq. KBE3)
// C^< = I^R + I^< + I^] is the lesser-form history sum of kbe_collision at (t_n,t_m), C^> the
// greater-form one (KBE_GREATER), J^] the Eq. KBE3 history terms, all on the self-energy row of
// kbe_sigma_2b, and eps the Fock matrix of Eq. eps for a local interaction with a Gaussian
// pulse on h_00:  eps = h0 + A exp(-(t-t0)^2 / (2 s^2)) e_00 + diag(-i u_i G^<_ii(t,t)).
// U_m and R_m are born at t_m (values kp[m][m] and -i; their derivatives there, "birth
// derivatives", come from the step that created them).
//
// Each element advances over [t_{n-1}, t_n] by the implicit Adams-Moulton rule in Lagrange form,
// y_n = y_{n-1} + sum_i lam_i f(t_{n-k+1+i}), with the local weights of Eq. weights on the nodes
// t_{n-k+1..n} (kbe_step_weights: the history integrals' rule of interval n) and k =
// min(order[n], n - b + 1) for an element born at t_b.  The implicit equation is solved by K
// fixed-point iterations from the explicit Euler predictor; the f values kept for later steps are
// evaluated once more at the accepted values (P (EC)^K E).
//
// Every step runs on the library's kernels: kbe_sigma_2b's row kernel, the collision kernels
// (lesser and greater form) and the small kernels below; the host only sequences launches on
// one stream.  The adjoint runs the steps backwards, recomputing the self-energy rows from the
// stored iterates and calling the collision and self-energy adjoints (kbe_collision_vjp,
// kbe_sigma_2b_vjp), so that d(loss)/du and d(loss)/dA of a loss on the densities
// n_i(t_n) = Re(-i G^<_ii(t_n,t_n)) are exact derivatives of the discrete map above.
#include <atomic>
#include <cmath>
#include <cstring>
#include <vector>

#include "kbe_dev.h"
#include "kbe_internal.h"

namespace kbe {
namespace {

constexpr int KM = KBE_KMAX;

// Element kinds of a step (index e in [0, 2n+1+ntau), then the two birth derivatives).
enum { EU = 0, ED = 1, ER = 2, ET = 3, EBU = 4, EBR = 5 };

struct PA {                       // everything the small kernels read, passed by value
  int N, nt, ntau, K;
  int64_t ldt;                    // row stride of the solution's kp (blocks)
  kbe_c128 *kp, *rdiag, *tv;      // the solution
  const kbe_c128 *mat;
  const double *h0, *u, *t, *lam;
  const int32_t *order;
  double amp, t0, sig;
  kbe_c128 *fkp, *fbu, *fbr, *ftv;  // f history (compact, row stride nt)
  kbe_c128 *ykp, *ytv;              // iterates y^(0..K) of each step's elements
  kbe_c128 *eps;                    // [E]
  kbe_c128 *IRl, *ILl, *Itv, *Jtv, *IRg, *ILg;  // history sums of the current evaluation
  kbe_c128 *base, *ynext;           // [elements][E]
  // adjoint
  kbe_c128 *gkp, *gtv;              // gradient of the solution (same layout as kp, tv)
  kbe_c128 *gfkp, *gfbu, *gfbr, *gftv;  // gradient of the f history
  kbe_c128 *ybar, *bbar, *fbar, *epart;  // [elements][E]
  kbe_c128 *epp;                          // [element chunks][E] partial sums of epart
  kbe_c128 *CbL, *CbG, *CbT, *Jbar;      // cotangents of the history sums
  kbe_c128 *gretL, *glesL, *gretG, *glesG;
  // adaptive propagation: one method order q for every element, rules of the current interval,
  // right sides of U_m / R_m below their birth (fpu[m][i], fpr[m][i]: at t_{m-1-i}, i < QM)
  int adaptive, q;
  const double *amt, *abt;          // [KM][KM]: corrector (k nodes) and predictor (q nodes) rules
  const double *wtau_;              // [ntau] the full-range tau rule
  kbe_c128 *fpu, *fpr;
};

constexpr int QM = 12;  // the largest Adams order of the adaptive propagation
constexpr int KSW = QM + 2;  // history orders recorded per step (at most maxcor + 1 evaluations)
// the collision outputs of the lesser form, and the greater form's I^R, I^< (Eq. KBE2)
constexpr unsigned FL = KBE_OUT_ALL;
constexpr unsigned FG = KBE_OUT_IR | KBE_OUT_IL | KBE_GREATER;

__device__ __forceinline__ int64_t E_(const PA &a) { return (int64_t)a.N * a.N; }
__device__ __forceinline__ int nelem(const PA &a, int n) { return 2 * n + 1 + a.ntau; }

__device__ __forceinline__ void elem_of(const PA &a, int n, int e, int &kind, int &idx) {
  const int ne = nelem(a, n);
  if (e < n) { kind = EU; idx = e; }
  else if (e == n) { kind = ED; idx = n; }
  else if (e <= 2 * n) { kind = ER; idx = e - n - 1; }
  else if (e < ne) { kind = ET; idx = e - 2 * n - 1; }
  else if (e == ne) { kind = EBU; idx = n; }
  else { kind = EBR; idx = n; }
}

__device__ __forceinline__ int birth(int kind, int idx) {
  return (kind == EU || kind == ER) ? idx : 0;
}

// Nodes of the rule of interval n for an element born at t_b (adaptive: the step's order, every
// element having a history of that length).
__device__ __forceinline__ int nodes(const PA &a, int n, int b) {
  if (a.adaptive) return a.q;
  int k = a.order[n];
  k = k < 1 ? 1 : (k > KM ? KM : k);
  return k < n - b + 1 ? k : n - b + 1;
}
__device__ __forceinline__ const double *lamrow(const PA &a, int n, int k) {
  if (a.adaptive) return a.amt + (int64_t)(k - 1) * KM;
  return a.lam + ((int64_t)n * KM + (k - 1)) * KM;
}

// The element's value at step n in the solution / in a gradient of the same layout.
__device__ __forceinline__ int64_t val_off(const PA &a, int n, int kind, int idx, bool tvarr) {
  (void)tvarr;
  switch (kind) {
    case EU: return ((int64_t)idx * a.ldt + n) * E_(a);
    case ED: return ((int64_t)n * a.ldt + n) * E_(a);
    case ER: return ((int64_t)n * a.ldt + idx) * E_(a);
    default: return ((int64_t)n * a.ntau + idx) * E_(a);  // ET: in tv
  }
}
__device__ __forceinline__ kbe_c128 *val_ptr(const PA &a, kbe_c128 *kp, kbe_c128 *tv, int n,
                                             int kind, int idx) {
  return (kind == ET ? tv : kp) + val_off(a, n, kind, idx, kind == ET);
}
// The element's iterate slot (compact layout, row stride nt).
__device__ __forceinline__ kbe_c128 *slot_ptr(const PA &a, int slot, int n, int kind, int idx) {
  const int64_t E = E_(a), nt = a.nt;
  if (kind == ET) return a.ytv + (((int64_t)slot * nt + n) * a.ntau + idx) * E;
  const int64_t base = (int64_t)slot * nt * nt;
  switch (kind) {
    case EU: return a.ykp + (base + (int64_t)idx * nt + n) * E;
    case ED: return a.ykp + (base + (int64_t)n * nt + n) * E;
    default: return a.ykp + (base + (int64_t)n * nt + idx) * E;  // ER
  }
}
// f of the element at step j (j >= its birth); the same layout for the f history and its
// gradient (pass the matching arrays).
__device__ __forceinline__ kbe_c128 *f_ptr(const PA &a, kbe_c128 *fkp, kbe_c128 *fbu,
                                           kbe_c128 *fbr, kbe_c128 *ftv, int j, int kind,
                                           int idx) {
  const int64_t E = E_(a), nt = a.nt;
  switch (kind) {
    case EU:
      if (j < idx) return a.fpu + ((int64_t)idx * QM + (idx - 1 - j)) * E;  // below its birth
      return j == idx ? fbu + idx * E : fkp + ((int64_t)idx * nt + j) * E;
    case ER:
      if (j < idx) return a.fpr + ((int64_t)idx * QM + (idx - 1 - j)) * E;
      return j == idx ? fbr + idx * E : fkp + ((int64_t)j * nt + idx) * E;
    case ED: return fkp + ((int64_t)j * nt + j) * E;
    case ET: return ftv + ((int64_t)j * a.ntau + idx) * E;
    case EBU: return fbu + (int64_t)j * E;
    default: return fbr + (int64_t)j * E;  // EBR
  }
}
// The element's value at t_{n-1} (its birth value for an element born there); nullptr for the
// constant -i (R_{n-1}, born on the diagonal).
__device__ __forceinline__ kbe_c128 *prev_ptr(const PA &a, kbe_c128 *kp, kbe_c128 *tv, int n,
                                              int kind, int idx) {
  const int64_t E = E_(a);
  switch (kind) {
    case EU: return kp + ((int64_t)idx * a.ldt + (n - 1)) * E;
    case ED: return kp + ((int64_t)(n - 1) * a.ldt + (n - 1)) * E;
    case ER: return idx < n - 1 ? kp + ((int64_t)(n - 1) * a.ldt + idx) * E : nullptr;
    default: return tv + ((int64_t)(n - 1) * a.ntau + idx) * E;
  }
}

__device__ __forceinline__ cd mul_i(cd z) { return {-z.im, z.re}; }    // i z
__device__ __forceinline__ cd mul_mi(cd z) { return {z.im, -z.re}; }   // -i z

__device__ __forceinline__ double pulse(const PA &a, int n) {
  const double d = a.t[n] - a.t0;
  return exp(-d * d / (2.0 * a.sig * a.sig));
}

// ---------------------------------------------------------------------------------------------
// Forward kernels
// ---------------------------------------------------------------------------------------------

// Initial state (Eq. BC): rdiag = -i 1 at every t; with a thermal branch
// G^](0,tau_j) = -i G^M(beta - tau_j) = -i mat[J-j] and G^<(0,0) = -G^](0,0)^dagger; without one
// kp[0][0] = G^<(0,0) is the caller's.
__global__ void prop_init(PA a) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nrd = (int64_t)a.nt * E;
  if (gid < nrd) {
    const int q = (int)(gid % E), r = q / a.N, c = q % a.N;
    st(a.rdiag + gid, {0.0, r == c ? -1.0 : 0.0});
    return;
  }
  if (a.ntau == 0) return;
  const int64_t g2 = gid - nrd;
  const int J = a.ntau - 1;
  if (g2 < (int64_t)a.ntau * E) {
    const int j = (int)(g2 / E), q = (int)(g2 % E);
    st(a.tv + g2, mul_mi(ld(a.mat + (int64_t)(J - j) * E + q)));
    if (j == 0) {  // kp[0][0][r][c] = -conj(tv[0][0][c][r]) = -i conj(mat[J][c][r])
      const int r = q / a.N, c = q % a.N;
      st(a.kp + (int64_t)r * a.N + c, mul_mi(cj(ld(a.mat + (int64_t)J * E + c * a.N + r))));
    }
  }
}

// eps(t_n) from the current G^<(t_n,t_n).
__global__ void prop_eps(PA a, int n) {
  const int q = threadIdx.x;
  const int64_t E = E_(a);
  if (q >= E) return;
  const int r = q / a.N, c = q % a.N;
  cd e = {a.h0[q], 0.0};
  if (r == 0 && c == 0) e.re += a.amp * pulse(a, n);
  if (r == c) {
    const cd d = ld(a.kp + ((int64_t)n * a.ldt + n) * E + (int64_t)r * a.N + r);
    e = e + a.u[r] * mul_mi(d);
  }
  st(a.eps + q, e);
}

// Adams-Moulton base sums and explicit Euler predictors of step n; the predictor becomes the
// current value of row/column n and iterate 0.
__global__ void prop_predict(PA a, int n) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nelem(a, n) * E) return;
  const int e = (int)(gid / E), q = (int)(gid % E);
  int kind, idx;
  elem_of(a, n, e, kind, idx);
  const int b = birth(kind, idx), k = nodes(a, n, b);
  const double *L = lamrow(a, n, k);
  const double h = a.t[n] - a.t[n - 1];
  const kbe_c128 *pp = prev_ptr(a, a.kp, a.tv, n, kind, idx);
  const int r = q / a.N, c = q % a.N;
  const cd prev = pp ? ld(pp + q) : cd{0.0, r == c ? -1.0 : 0.0};
  cd base = prev;
  for (int i = 0; i + 1 < k; ++i)
    base = base + L[i] * ld(f_ptr(a, a.fkp, a.fbu, a.fbr, a.ftv, n - k + 1 + i, kind, idx) + q);
  const cd pred = prev + h * ld(f_ptr(a, a.fkp, a.fbu, a.fbr, a.ftv, n - 1, kind, idx) + q);
  st(a.base + gid, base);
  st(val_ptr(a, a.kp, a.tv, n, kind, idx) + q, pred);
  st(slot_ptr(a, 0, n, kind, idx) + q, pred);
}

// f of every element of step n at the current values.  mode 0: the next iterate base +
// lam_last f into ynext; mode 1: the f history at t_n, birth derivatives included.
__global__ void prop_rhs(PA a, int n, int mode) {
  const int64_t E = E_(a);
  const int N = a.N;
  const int ne = nelem(a, n) + (mode ? 2 : 0);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)ne * E) return;
  const int e = (int)(gid / E), q = (int)(gid % E), r = q / N, c = q % N;
  int kind, idx;
  elem_of(a, n, e, kind, idx);
  const bool th = a.ntau > 0;
  auto Cl = [&](int m, int rr, int cc) {
    const int64_t o = (int64_t)m * E + rr * N + cc;
    cd s = ld(a.IRl + o) + ld(a.ILl + o);
    return th ? s + ld(a.Itv + o) : s;
  };
  auto Cg = [&](int m, int rr, int cc) {
    const int64_t o = (int64_t)m * E + rr * N + cc;
    cd s = ld(a.IRg + o) + ld(a.ILg + o);
    return th ? s + ld(a.Itv + o) : s;
  };
  const kbe_c128 *ep = a.eps;
  cd f = czero();
  if (kind == EU || kind == EBU) {  // i (X eps - C^<(n,m)^dagger)
    const int m = kind == EU ? idx : n;
    const kbe_c128 *X = a.kp + ((int64_t)m * a.ldt + n) * E;
    cd s = czero();
#pragma unroll 8
    for (int k = 0; k < N; ++k) s = s + ld(X + r * N + k) * ld(ep + k * N + c);
    f = mul_i(s - cj(Cl(m, c, r)));
  } else if (kind == ER) {  // -i (eps X + C^> - C^<)
    const kbe_c128 *X = a.kp + ((int64_t)n * a.ldt + idx) * E;
    cd s = czero();
#pragma unroll 8
    for (int k = 0; k < N; ++k) s = s + ld(ep + r * N + k) * ld(X + k * N + c);
    f = mul_mi(s + Cg(idx, r, c) - Cl(idx, r, c));
  } else if (kind == EBR) {  // -i (eps (-i 1) + C^>(n,n) - C^<(n,n))
    f = mul_mi(mul_mi(ld(ep + q)) + Cg(n, r, c) - Cl(n, r, c));
  } else if (kind == ED) {  // -i [eps, D] - i (C + C^dagger)
    const kbe_c128 *X = a.kp + ((int64_t)n * a.ldt + n) * E;
    cd s = czero();
    for (int k = 0; k < N; ++k)
      s = s + ld(ep + r * N + k) * ld(X + k * N + c) - ld(X + r * N + k) * ld(ep + k * N + c);
    f = mul_mi(s + Cl(n, r, c) + cj(Cl(n, c, r)));
  } else {  // ET: -i (eps X + J)
    const kbe_c128 *X = a.tv + ((int64_t)n * a.ntau + idx) * E;
    cd s = czero();
#pragma unroll 8
    for (int k = 0; k < N; ++k) s = s + ld(ep + r * N + k) * ld(X + k * N + c);
    f = mul_mi(s + ld(a.Jtv + (int64_t)idx * E + q));
  }
  if (mode == 0) {
    const int k = nodes(a, n, birth(kind, idx));
    st(a.ynext + gid, ld(a.base + gid) + lamrow(a, n, k)[k - 1] * f);
  } else {
    st(f_ptr(a, a.fkp, a.fbu, a.fbr, a.ftv, n, kind, idx) + q, f);
  }
}

// The next iterate becomes the current value of row/column n and iterate `slot`.
__global__ void prop_commit(PA a, int n, int slot) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nelem(a, n) * E) return;
  const int e = (int)(gid / E), q = (int)(gid % E);
  int kind, idx;
  elem_of(a, n, e, kind, idx);
  const cd y = ld(a.ynext + gid);
  st(val_ptr(a, a.kp, a.tv, n, kind, idx) + q, y);
  if (slot >= 0) st(slot_ptr(a, slot, n, kind, idx) + q, y);
}

// Row/column n from iterate `slot` (adjoint: the values an evaluation saw).
__global__ void prop_restore(PA a, int n, int slot) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nelem(a, n) * E) return;
  const int e = (int)(gid / E), q = (int)(gid % E);
  int kind, idx;
  elem_of(a, n, e, kind, idx);
  st(val_ptr(a, a.kp, a.tv, n, kind, idx) + q, ld(slot_ptr(a, slot, n, kind, idx) + q));
}

__global__ void prop_dens(PA a, int n, double *dens) {
  const int r = threadIdx.x;
  if (r >= a.N) return;
  const cd d = ld(a.kp + ((int64_t)n * a.ldt + n) * E_(a) + (int64_t)r * a.N + r);
  dens[(int64_t)n * a.N + r] = d.im;  // Re(-i d)
}

// ---------------------------------------------------------------------------------------------
// Adjoint kernels (PyTorch's complex convention: a real loss L has the gradient dL/dRe + i dL/dIm;
// for y = a X b the cotangents are conj(a)^T ybar b^dagger ... written out per term below)
// ---------------------------------------------------------------------------------------------

template <typename T>
__global__ void fill_zero(T *p, int64_t count) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < count) p[gid] = T{};
}

// The loss's cotangent: d n_i(t_n) / d G^<_ii(t_n,t_n) pairs with i gdens[n][i].
__global__ void prop_seed(PA a, const double *gdens) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)a.nt * a.N) return;
  const int n = (int)(gid / a.N), r = (int)(gid % a.N);
  kbe_c128 *g = a.gkp + ((int64_t)n * a.ldt + n) * E_(a) + (int64_t)r * a.N + r;
  st(g, ld(g) + cd{0.0, gdens[gid]});
}

// fbar of the final evaluation of step n: the gradient of the stored f history at t_n.
__global__ void prop_gather_final(PA a, int n) {
  const int64_t E = E_(a);
  const int ne = nelem(a, n) + 2;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)ne * E) return;
  const int e = (int)(gid / E), q = (int)(gid % E);
  int kind, idx;
  elem_of(a, n, e, kind, idx);
  st(a.fbar + gid, ld(f_ptr(a, a.gfkp, a.gfbu, a.gfbr, a.gftv, n, kind, idx) + q));
}

// Cotangents of the history sums from fbar: C^<(m), C^>(m) (m <= n), I^] (both forms), J^](j).
__global__ void prop_cot(PA a, int n, int mode) {
  const int64_t E = E_(a);
  const int N = a.N;
  const int ne = nelem(a, n);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nm = (int64_t)(n + 1) * E;
  if (gid >= nm + (int64_t)a.ntau * E) return;
  const int q = (int)(gid % E), r = q / N, c = q % N;
  const int tq = c * N + r;  // transposed entry
  if (gid < nm) {
    const int m = (int)(gid / E);
    cd cl, cg;
    if (m < n) {
      const kbe_c128 *fu = a.fbar + (int64_t)m * E, *fr = a.fbar + (int64_t)(n + 1 + m) * E;
      cl = mul_mi(cj(ld(fu + tq))) + mul_mi(ld(fr + q));
      cg = mul_i(ld(fr + q));
    } else {
      const kbe_c128 *fd = a.fbar + (int64_t)n * E;
      cl = mul_i(ld(fd + q)) + mul_mi(cj(ld(fd + tq)));
      cg = czero();
      if (mode) {
        const kbe_c128 *fbu = a.fbar + (int64_t)ne * E, *fbr = a.fbar + (int64_t)(ne + 1) * E;
        cl = cl + mul_mi(cj(ld(fbu + tq))) + mul_mi(ld(fbr + q));
        cg = mul_i(ld(fbr + q));
      }
    }
    st(a.CbL + gid, cl);
    st(a.CbG + gid, cg);
    st(a.CbT + gid, cl + cg);
  } else {
    const int64_t g2 = gid - nm;
    const int j = (int)(g2 / E);
    st(a.Jbar + g2, mul_i(ld(a.fbar + (int64_t)(2 * n + 1 + j) * E + q)));
  }
}

// The terms of f that multiply the element itself or eps: their gradient into the solution's
// gradient (row/column n) and each element's share of the gradient of eps (epart[e]).
__global__ void prop_direct(PA a, int n, int mode) {
  const int64_t E = E_(a);
  const int N = a.N;
  const int ne = nelem(a, n);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)ne * E) return;
  const int e = (int)(gid / E), q = (int)(gid % E), r = q / N, c = q % N;
  int kind, idx;
  elem_of(a, n, e, kind, idx);
  const kbe_c128 *ep = a.eps;
  const kbe_c128 *fb = a.fbar + (int64_t)e * E;
  const kbe_c128 *X = val_ptr(a, a.kp, a.tv, n, kind, idx);
  kbe_c128 *gX = val_ptr(a, a.gkp, a.gtv, n, kind, idx);
  cd gx = czero(), ge = czero();
  if (kind == EU) {  // y = i X eps: Xbar += -i ybar eps^H, epsbar += -i X^H ybar
    for (int k = 0; k < N; ++k) {
      gx = gx + ld(fb + r * N + k) * cj(ld(ep + c * N + k));
      ge = ge + cj(ld(X + k * N + r)) * ld(fb + k * N + c);
    }
    gx = mul_mi(gx);
    ge = mul_mi(ge);
  } else if (kind == ER || kind == ET) {  // y = -i eps X: Xbar += i eps^H ybar, epsbar += i ybar X^H
    for (int k = 0; k < N; ++k) {
      gx = gx + cj(ld(ep + k * N + r)) * ld(fb + k * N + c);
      ge = ge + ld(fb + r * N + k) * cj(ld(X + c * N + k));
    }
    gx = mul_i(gx);
    ge = mul_i(ge);
  } else {  // ED: y = -i eps D + i D eps (+ birth of U_n: i D eps; of R_n: -eps)
    cd a1 = czero(), a2 = czero(), b1 = czero(), b2 = czero();
    for (int k = 0; k < N; ++k) {
      a1 = a1 + cj(ld(ep + k * N + r)) * ld(fb + k * N + c);  // eps^H ybar
      a2 = a2 + ld(fb + r * N + k) * cj(ld(ep + c * N + k));  // ybar eps^H
      b1 = b1 + ld(fb + r * N + k) * cj(ld(X + c * N + k));   // ybar D^H
      b2 = b2 + cj(ld(X + k * N + r)) * ld(fb + k * N + c);   // D^H ybar
    }
    gx = mul_i(a1) + mul_mi(a2);
    ge = mul_i(b1) + mul_mi(b2);
    if (mode) {
      const kbe_c128 *fu = a.fbar + (int64_t)ne * E, *fr = a.fbar + (int64_t)(ne + 1) * E;
      cd a3 = czero(), b3 = czero();
      for (int k = 0; k < N; ++k) {
        a3 = a3 + ld(fu + r * N + k) * cj(ld(ep + c * N + k));  // ybar_bu eps^H
        b3 = b3 + cj(ld(X + k * N + r)) * ld(fu + k * N + c);   // D^H ybar_bu
      }
      gx = gx + mul_mi(a3);
      ge = ge + mul_mi(b3) - ld(fr + q);
    }
  }
  st(gX + q, ld(gX + q) + gx);
  st(a.epart + gid, ge);
}

// epsbar = sum of the element shares (fixed order), then through eps: the Fock term into
// G^<(t_n,t_n) and u, the pulse into its amplitude.
// eps's gradient: the per-element shares summed in a fixed order, in two stages (chunks of
// EPC elements over many workgroups, then the chunks in order).
constexpr int EPC = 32;
__global__ void prop_eps_part(PA a, int n) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ne = nelem(a, n), nch = (ne + EPC - 1) / EPC;
  if (gid >= (int64_t)nch * E) return;
  const int ch = (int)(gid / E), q = (int)(gid % E);
  const int e1 = (ch + 1) * EPC < ne ? (ch + 1) * EPC : ne;
  cd s = czero();
#pragma unroll 8
  for (int e = ch * EPC; e < e1; ++e) s = s + ld(a.epart + (int64_t)e * E + q);  // loads issued together, added in order
  st(a.epp + gid, s);
}

__global__ void prop_eps_vjp(PA a, int n, double *gu, double *gamp) {
  const int64_t E = E_(a);
  const int q = threadIdx.x;
  if (q >= E) return;
  const int nch = (nelem(a, n) + EPC - 1) / EPC;
  cd s = czero();
#pragma unroll 8
  for (int ch = 0; ch < nch; ++ch) s = s + ld(a.epp + (int64_t)ch * E + q);  // added in order
  const int r = q / a.N, c = q % a.N;
  if (r == c) {  // eps_rr += -i u_r D_rr
    kbe_c128 *g = a.gkp + ((int64_t)n * a.ldt + n) * E + q;
    const cd d = ld(a.kp + ((int64_t)n * a.ldt + n) * E + q);
    st(g, ld(g) + a.u[r] * mul_i(s));
    const cd w = mul_mi(d);  // d eps_rr / d u_r
    gu[r] += w.re * s.re + w.im * s.im;
  }
  if (q == 0) gamp[0] += pulse(a, n) * s.re;
}

// gS = gS(lesser) + gS(greater) over the real-time row.
__global__ void prop_gs_add(PA a, int n) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)(n + 1) * E_(a)) return;
  st(a.gretL + gid, ld(a.gretL + gid) + ld(a.gretG + gid));
  st(a.glesL + gid, ld(a.glesL + gid) + ld(a.glesG + gid));
}

// ybar of iterate `it` (the gradient accumulated in row/column n), reset for the next; the
// base's gradient accumulates it, and fbar = lam_last ybar feeds the evaluation that made it.
__global__ void prop_take(PA a, int n, int first) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nelem(a, n) * E) return;
  const int e = (int)(gid / E), q = (int)(gid % E);
  int kind, idx;
  elem_of(a, n, e, kind, idx);
  kbe_c128 *g = val_ptr(a, a.gkp, a.gtv, n, kind, idx) + q;
  const cd y = ld(g);
  st(g, czero());
  st(a.bbar + gid, first ? y : ld(a.bbar + gid) + y);
  const int k = nodes(a, n, birth(kind, idx));
  st(a.fbar + gid, lamrow(a, n, k)[k - 1] * y);
}

// Predictor and base sums of step n, backwards: the gradient of iterate 0 (left in row/column
// n) and of the base reach the values at t_{n-1} and the f history of the rule's nodes.
__global__ void prop_predict_vjp(PA a, int n) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nelem(a, n) * E) return;
  const int e = (int)(gid / E), q = (int)(gid % E);
  int kind, idx;
  elem_of(a, n, e, kind, idx);
  const cd y0 = ld(val_ptr(a, a.gkp, a.gtv, n, kind, idx) + q);
  const cd bb = ld(a.bbar + gid);
  const double h = a.t[n] - a.t[n - 1];
  // values at t_{n-1}; U_{n-1}'s is G^<(t_{n-1},t_{n-1}), D's too: D's thread adds both
  if (!(kind == EU && idx == n - 1)) {
    kbe_c128 *gp = prev_ptr(a, a.gkp, a.gtv, n, kind, idx);
    if (gp) {
      cd add = y0 + bb;
      if (kind == ED && n - 1 >= 0) {
        const int64_t eu = (int64_t)(n - 1) * E + q;  // element U_{n-1}
        add = add + ld(val_ptr(a, a.gkp, a.gtv, n, EU, n - 1) + q) + ld(a.bbar + eu);
      }
      st(gp + q, ld(gp + q) + add);
    }
  }
  const int b = birth(kind, idx), k = nodes(a, n, b);
  const double *L = lamrow(a, n, k);
  for (int i = 0; i + 1 < k; ++i) {
    const int j = n - k + 1 + i;
    kbe_c128 *gf = f_ptr(a, a.gfkp, a.gfbu, a.gfbr, a.gftv, j, kind, idx) + q;
    cd add = L[i] * bb;
    if (j == n - 1) add = add + h * y0;
    st(gf, ld(gf) + add);
  }
  if (k == 1) {  // the rule has no history node: the predictor's f at t_{n-1} only
    kbe_c128 *gf = f_ptr(a, a.gfkp, a.gfbu, a.gfbr, a.gftv, n - 1, kind, idx) + q;
    st(gf, ld(gf) + h * y0);
  }
}

// ---------------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------------
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t fkp, fbu, fbr, ftv, ykp, ytv, eps, sig_ret, sig_les, sig_tv, IRl, ILl, Itv, Jtv, IRg,
      ILg, base, ynext, cws;                                  // forward
  size_t gkp, grd, gtv, gmat, gfkp, gfbu, gfbr, gftv, ybar, bbar, fbar, epart, epp, CbL, CbG, CbT,
      Jbar, gretL, glesL, gstvL, gretG, glesG, gstvG, vws, sws;  // adjoint
  size_t total;
};

Layout layout(int N, int nt, int ntau, int64_t ldt, int K) {
  const size_t E = (size_t)N * N * sizeof(kbe_c128);
  const size_t nt2 = (size_t)nt * nt, ne = (size_t)(2 * nt + 1 + ntau + 2);
  const int n = nt - 1;
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t r = o; o += al(bytes); return r; };
  L.fkp = take(nt2 * E);
  L.fbu = take(nt * E);
  L.fbr = take(nt * E);
  L.ftv = take((size_t)nt * ntau * E);
  L.ykp = take((size_t)(K + 1) * nt2 * E);
  L.ytv = take((size_t)(K + 1) * nt * ntau * E);
  L.eps = take(E);
  L.sig_ret = take(nt * E);
  L.sig_les = take(nt * E);
  L.sig_tv = take(ntau * E);
  L.IRl = take(nt * E);
  L.ILl = take(nt * E);
  L.Itv = take(nt * E);
  L.Jtv = take(ntau * E);
  L.IRg = take(nt * E);
  L.ILg = take(nt * E);
  L.base = take(ne * E);
  L.ynext = take(ne * E);
  L.cws = take(collision_ws_bytes_rows(N, nt, ntau, KBE_OUT_ALL | KBE_INT_BOTH));
  L.gkp = take((size_t)nt * ldt * E);
  L.grd = take(nt * E);
  L.gtv = take((size_t)nt * ntau * E);
  L.gmat = take(ntau * E);
  L.gfkp = take(nt2 * E);
  L.gfbu = take(nt * E);
  L.gfbr = take(nt * E);
  L.gftv = take((size_t)nt * ntau * E);
  L.ybar = take(ne * E);
  L.bbar = take(ne * E);
  L.fbar = take(ne * E);
  L.epart = take(ne * E);
  L.epp = take(((ne + EPC - 1) / EPC) * E);
  L.CbL = take(nt * E);
  L.CbG = take(nt * E);
  L.CbT = take(nt * E);
  L.Jbar = take(ntau * E);
  L.gretL = take(nt * E);
  L.glesL = take(nt * E);
  L.gstvL = take(ntau * E);
  L.gretG = take(nt * E);
  L.glesG = take(nt * E);
  L.gstvG = take(ntau * E);
  size_t vw = collision_vjp_ws_bytes_rows(N, nt, ntau, KBE_OUT_ALL);
  const size_t vw2 = collision_vjp_ws_bytes_rows(N, nt, ntau, FG | KBE_INT_GREXTRA);
  L.vws = take(vw > vw2 ? vw : vw2);
  L.sws = take(sigma_vjp_ws_bytes(N, n, ntau));
  L.total = o;
  return L;
}

struct Ctx {
  PA a;
  Layout L;
  char *ws;
  const kbe_green *G;
  const kbe_wts *W;
  kbe_green Gc;          // the solution as a kbe_green (for the Sigma and collision calls)
  kbe_green gG;          // its gradient (adjoint)
  kbe_sigma_row sig, gSL, gSG;
  hipStream_t st;
};

unsigned blocks(int64_t count) { return (unsigned)((count + 255) / 256); }

Params coll_params(const Ctx &x, int n) {
  Params p{};
  p.N = x.a.N;
  p.nt = x.a.nt;
  p.ntau = x.a.ntau;
  p.J = x.a.ntau - 1;
  p.n = n;
  p.m0 = 0;
  p.m1 = n + 1;
  p.ldt = x.a.ldt;
  p.kp = x.a.kp;
  p.rdiag = x.a.rdiag;
  p.tv = x.a.tv;
  p.mat = x.a.mat;
  p.ret = x.sig.ret;
  p.les = x.sig.les;
  p.stv = x.sig.tv;
  p.w = x.W->w;
  p.wtau = x.W->wtau;
  p.wf = x.W->wtau_fwd;
  return p;
}

void set_flags(Params &p, unsigned flags, bool th) {
  p.fIR = (flags & KBE_OUT_IR) != 0;
  p.fIL = (flags & KBE_OUT_IL) != 0;
  p.fITV = (flags & KBE_OUT_ITV) && th;
  p.fJTV = (flags & KBE_OUT_JTV) && th;
  p.overwrite = 0;
}


// Self-energy row and both history sums of step n at the current values, then eps.
hipError_t evaluate(Ctx &x, int n) {
  hipError_t e = launch_sigma_row(&x.Gc, x.a.u, n, &x.sig, x.st);
  if (e != hipSuccess) return e;
  const bool th = x.a.ntau > 0;
  Params p = coll_params(x, n);
  set_flags(p, FL, th);
  e = launch_collision_both(p, x.a.IRl, x.a.ILl, x.a.Itv, x.a.Jtv, x.a.IRg, x.a.ILg,
                            x.ws + x.L.cws, x.st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prop_eps, dim3(1), dim3(256), 0, x.st, x.a, n);
  return hipGetLastError();
}

// The adjoint of one evaluation at the current values, given fbar: eps, sums and Sigma row.
hipError_t evaluate_vjp(Ctx &x, int n, int mode, double *gu, double *gamp) {
  hipError_t e = launch_sigma_row(&x.Gc, x.a.u, n, &x.sig, x.st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prop_eps, dim3(1), dim3(256), 0, x.st, x.a, n);
  const int64_t E = (int64_t)x.a.N * x.a.N;
  const int ne = 2 * n + 1 + x.a.ntau;
  hipLaunchKernelGGL(prop_cot, dim3(blocks((int64_t)(n + 1 + x.a.ntau) * E)), dim3(256), 0, x.st,
                     x.a, n, mode);
  hipLaunchKernelGGL(prop_direct, dim3(blocks((int64_t)ne * E)), dim3(256), 0, x.st, x.a, n, mode);
  const int64_t nch = (ne + EPC - 1) / EPC;
  hipLaunchKernelGGL(prop_eps_part, dim3(blocks(nch * E)), dim3(256), 0, x.st, x.a, n);
  hipLaunchKernelGGL(prop_eps_vjp, dim3(1), dim3(256), 0, x.st, x.a, n, gu, gamp);
  const bool th = x.a.ntau > 0;
  Params p = coll_params(x, n);
  p.gkp = x.gG.kp;
  p.grdiag = x.gG.rdiag;
  p.gtv = x.gG.tv;
  // Both forms by linearity: the lesser form's adjoint with the summed cotangents (the terms
  // the forms share, I^R's and the Sigma^< part of I^<, enter C^< and C^> alike, as I^] does:
  // CbT = CbL + CbG), then the greater form's further terms with its own cotangent.
  Params pg = p;
  set_flags(p, FL, th);
  p.gIR = x.a.CbT;
  p.gIL = x.a.CbT;
  p.gItv = x.a.CbT;
  p.gJ = x.a.Jbar;
  set_flags(pg, FG, th);
  pg.gIR = x.a.CbG;
  pg.gIL = x.a.CbG;
  pg.gItv = nullptr;
  pg.gJ = nullptr;
  e = launch_collision_vjp_pair(p, FL, pg, FG | KBE_INT_GREXTRA, x.gG.mat, &x.gSL, &x.gSG,
                                x.ws + x.L.vws, x.st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prop_gs_add, dim3(blocks((int64_t)(n + 1) * E)), dim3(256), 0, x.st, x.a, n);
  return launch_sigma_row_vjp(&x.Gc, x.a.u, n, &x.gSL, &x.gG, gu, x.ws + x.L.sws, x.st);
}

Ctx make_ctx(const kbe_prop *P, const kbe_wts *W, const kbe_green *G, void *ws, hipStream_t st) {
  Ctx x{};
  x.L = layout(G->N, G->nt, G->ntau, G->ldt, P->iters);
  x.ws = (char *)ws;
  x.G = G;
  x.W = W;
  x.st = st;
  x.Gc = *G;
  PA &a = x.a;
  a.N = G->N;
  a.nt = G->nt;
  a.ntau = G->ntau;
  a.K = P->iters;
  a.ldt = G->ldt;
  a.kp = G->kp;
  a.rdiag = G->rdiag;
  a.tv = G->tv;
  a.mat = G->mat;
  a.h0 = P->h0;
  a.u = P->u;
  a.t = P->t;
  a.lam = P->lam;
  a.order = P->order;
  a.amp = P->pulse_amp;
  a.t0 = P->pulse_t0;
  a.sig = P->pulse_sigma;
  auto c = [&](size_t off) { return (kbe_c128 *)(x.ws + off); };
  a.fkp = c(x.L.fkp);
  a.fbu = c(x.L.fbu);
  a.fbr = c(x.L.fbr);
  a.ftv = c(x.L.ftv);
  a.ykp = c(x.L.ykp);
  a.ytv = c(x.L.ytv);
  a.eps = c(x.L.eps);
  a.IRl = c(x.L.IRl);
  a.ILl = c(x.L.ILl);
  a.Itv = c(x.L.Itv);
  a.Jtv = c(x.L.Jtv);
  a.IRg = c(x.L.IRg);
  a.ILg = c(x.L.ILg);
  a.base = c(x.L.base);
  a.ynext = c(x.L.ynext);
  a.gkp = c(x.L.gkp);
  a.gtv = c(x.L.gtv);
  a.gfkp = c(x.L.gfkp);
  a.gfbu = c(x.L.gfbu);
  a.gfbr = c(x.L.gfbr);
  a.gftv = c(x.L.gftv);
  a.ybar = c(x.L.ybar);
  a.bbar = c(x.L.bbar);
  a.fbar = c(x.L.fbar);
  a.epart = c(x.L.epart);
  a.epp = c(x.L.epp);
  a.CbL = c(x.L.CbL);
  a.CbG = c(x.L.CbG);
  a.CbT = c(x.L.CbT);
  a.Jbar = c(x.L.Jbar);
  a.gretL = c(x.L.gretL);
  a.glesL = c(x.L.glesL);
  a.gretG = c(x.L.gretG);
  a.glesG = c(x.L.glesG);
  x.sig = {c(x.L.sig_ret), c(x.L.sig_les), a.ntau ? c(x.L.sig_tv) : nullptr};
  x.gSL = {a.gretL, a.glesL, a.ntau ? c(x.L.gstvL) : nullptr};
  x.gSG = {a.gretG, a.glesG, a.ntau ? c(x.L.gstvG) : nullptr};
  x.gG = *G;
  x.gG.kp = a.gkp;
  x.gG.rdiag = c(x.L.grd);
  x.gG.tv = a.ntau ? a.gtv : nullptr;
  x.gG.mat = a.ntau ? c(x.L.gmat) : nullptr;
  return x;
}

// ---------------------------------------------------------------------------------------------
// Adaptive propagation (Sec. "Adaptive Time Stepping", Sec. "Adaptive History Integration"):
// the kernels of a step; the controller is host code below.
// ---------------------------------------------------------------------------------------------
struct AA {                        // adaptive-only arrays
  double *t;                       // [nt] the grid (device copy, written point by point)
  double *w;                       // [nt][nt] history weights, built row by row
  kbe_c128 *ypred;                 // [elements][E] predictor values
  kbe_c128 *sret, *sles, *stv;     // Sigma rows of the current evaluation
  kbe_c128 *Sret, *Sles, *Stv;     // Sigma rows of every accepted step [nt][nt], [nt][ntau]
  kbe_c128 *epsall;                // [nt][E] eps of every accepted step
  kbe_c128 *ubuf;                  // [KM][E] test-integrand values
  kbe_c128 *Cl, *Cg;               // [QM][E] history sums above the diagonal
  kbe_c128 *upart;                 // [chunks][QM][2][E] their partial sums by term chunk
  double *part;                    // [2][NPART] norm partial sums
  uint32_t *done;                  // workgroups of a norm launch that have stored their partials
  uint32_t *cdone;                 // workgroups of an ad_choose launch that have stored their u
  double *res;                     // [2] norm results, in page-locked host memory
  volatile uint32_t *flag;         // sequence number of the last norm launch (host memory)
  int32_t *kbuf;                   // [nt][QM + 2] history order of every evaluation of each step
  double rtol, atol;
};

constexpr int NPART = 1024;  // workgroups of a norm launch, at most (each fences and counts once)

__global__ void ad_set_t(double *t, int n, double v) {
  if (threadIdx.x == 0) t[n] = v;
}

// Adams base sums (corrector history part) and predictors of step n at order a.q; the predictor
// becomes the current value of row/column n.
__global__ void ad_predict(PA a, AA b, int n) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nelem(a, n) * E) return;
  const int e = (int)(gid / E), q = (int)(gid % E);
  int kind, idx;
  elem_of(a, n, e, kind, idx);
  const int k = a.q;
  const double *L = a.amt + (int64_t)(k - 1) * KM, *B = a.abt + (int64_t)(k - 1) * KM;
  const kbe_c128 *pp = prev_ptr(a, a.kp, a.tv, n, kind, idx);
  const int r = q / a.N, c = q % a.N;
  const cd prev = pp ? ld(pp + q) : cd{0.0, r == c ? -1.0 : 0.0};
  cd base = prev, pred = prev;
  for (int i = 0; i + 1 < k; ++i)
    base = base + L[i] * ld(f_ptr(a, a.fkp, a.fbu, a.fbr, a.ftv, n - k + 1 + i, kind, idx) + q);
  for (int i = 0; i < k; ++i)
    pred = pred + B[i] * ld(f_ptr(a, a.fkp, a.fbu, a.fbr, a.ftv, n - k + i, kind, idx) + q);
  st(a.base + gid, base);
  st(b.ypred + gid, pred);
  st(val_ptr(a, a.kp, a.tv, n, kind, idx) + q, pred);
}

// The history order of interval n (Sec. "Adaptive History Integration"): the test integrand
// u(t_s) = G^R(t_n,t_s) Sigma^<(t_s,t_n) + G^<(t_n,t_s) Sigma^A(t_s,t_n) at s = n-K+1..n
// (Sigma^<(t_s,t_n) = -Sigma^<(t_n,t_s)^dagger, Sigma^A(t_s,t_n) = Sigma^R(t_n,t_s)^dagger,
// G^<(t_n,t_s) = -kp[s][n]^dagger), its integrals I^(k) over the interval with k = 1..K nodes,
// k_opt = the first minimum of ||I^(k) - I^(k-1)||_F over k = 2..K, and row n of the history
// weights: row n-1 plus the local weights on k_opt nodes.  The entries of u are spread over
// workgroups; the last one to finish (a counter it resets) makes the choice; fixed-order sums.
__global__ void __launch_bounds__(256) ad_choose(PA a, AA b, int n, int K, int64_t slot) {
  const int64_t E = E_(a);
  const int N = a.N;
  __shared__ double dk[KM + 1];
  __shared__ int kopt;
  __shared__ bool last;
  const int tid = threadIdx.x;
  // every workgroup computes 256 entries of u; the last one to finish chooses k_opt
  for (int64_t x = (int64_t)blockIdx.x * 256 + tid; x < (int64_t)K * E; x += (int64_t)gridDim.x * 256) {
    const int i = (int)(x / E), q = (int)(x % E), r = q / N, c = q % N;
    const int sidx = n - K + 1 + i;
    const kbe_c128 *gr = sidx < n ? a.kp + ((int64_t)n * a.ldt + sidx) * E : a.rdiag + n * E;
    const kbe_c128 *gl = a.kp + ((int64_t)sidx * a.ldt + n) * E;  // G^<(t_n,t_s) = -gl^dagger
    const kbe_c128 *sl = b.sles + sidx * E, *sr = b.sret + sidx * E;
    cd acc = czero();
#pragma unroll 8
    for (int k = 0; k < N; ++k) {  // unrolled: the loads of several k are issued together
      acc = acc - ld(gr + r * N + k) * cj(ld(sl + c * N + k));   // G^R (-Sigma^<^dagger)
      // G^<(t_n,t_s): -kp[s][n]^dagger, or kp[n][n] itself on the diagonal
      const cd g = sidx < n ? -cj(ld(gl + k * N + r)) : ld(gl + r * N + k);
      acc = acc + g * cj(ld(sr + c * N + k));                      // G^< Sigma^R^dagger
    }
    st(b.ubuf + x, acc);
  }
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    last = atomicAdd(b.cdone, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (tid == 0) *b.cdone = 0u;
  // ||I^(k) - I^(k-1)||_F for k = 2..K: wave w takes k = 2 + w, 6 + w, ...; each lane sums its
  // entries q = lane, lane + 64, ... and the wave sums the lanes by a fixed butterfly
  const int wave = tid / 64, lane = tid % 64;
  for (int k = 2 + wave; k <= K; k += 4) {
    double part = 0.0;
    const double *Lk = a.amt + (int64_t)(k - 1) * KM, *Lk1 = a.amt + (int64_t)(k - 2) * KM;
    for (int64_t q = lane; q < E; q += 64) {
      cd ik = czero(), ik1 = czero();
#pragma unroll 4
      for (int i = 0; i < k; ++i) ik = ik + Lk[i] * ld(b.ubuf + (int64_t)(K - k + i) * E + q);
#pragma unroll 4
      for (int i = 0; i < k - 1; ++i) ik1 = ik1 + Lk1[i] * ld(b.ubuf + (int64_t)(K - k + 1 + i) * E + q);
      const cd d = ik - ik1;
      part += d.re * d.re + d.im * d.im;
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if (lane == 0) dk[k] = sqrt(part);
  }
  __syncthreads();
  if (tid == 0) {
    int best = 2;
    for (int k = 3; k <= K; ++k)
      if (dk[k] < dk[best]) best = k;
    kopt = best;
    b.kbuf[slot] = best;
  }
  __syncthreads();
  const int k = kopt, lo = n - k + 1;
  const double *L = a.amt + (int64_t)(k - 1) * KM;
  for (int sidx = tid; sidx <= n; sidx += 256) {  // entries beyond n stay zero
    double v = sidx < n ? b.w[(int64_t)(n - 1) * a.nt + sidx] : 0.0;
    if (sidx >= lo && sidx <= n) v += L[sidx - lo];
    b.w[(int64_t)n * a.nt + sidx] = v;
  }
}

// Weighted root-mean-square norms over the entries of step n's elements (Eq. wrms_norm), with the
// weights of Eq. ewt from the values at t_{n-1}.  Up to two norms per launch (job j = 0, 1):
// kind 0: ynext - current; 1: C (current - predictor); 2: coef * f[t_{n-npts+1}..t_n] (a divided
// difference of every element's right sides); 3: C (ynext - predictor).  Each workgroup stores
// its partial sums; the last one to finish (a counter) sums the partials in workgroup order,
// writes the norms to b.res[j] and then the launch's sequence number to b.flag (page-locked host
// memory, which the controller polls), and resets the counter for the next launch.
struct NormJob {
  int kind, npts;
  double C, coef;
};

__device__ __forceinline__ cd norm_term(const PA &a, const AA &b, int n, int e, int q,
                                        int kind_e, int idx, int64_t gid, const NormJob &j) {
  if (j.kind == 0) return ld(a.ynext + gid) - ld(val_ptr(a, a.kp, a.tv, n, kind_e, idx) + q);
  if (j.kind == 1) return j.C * (ld(val_ptr(a, a.kp, a.tv, n, kind_e, idx) + q) - ld(b.ypred + gid));
  if (j.kind == 3) return j.C * (ld(a.ynext + gid) - ld(b.ypred + gid));
  // Newton's recursion over a fixed bound, predicated on npts, so the arrays stay in registers
  cd d[QM + 2];
  double tt[QM + 2];
#pragma unroll
  for (int i = 0; i < QM + 2; ++i) {
    if (i < j.npts) {
      const int jj = n - j.npts + 1 + i;
      tt[i] = b.t[jj];
      d[i] = ld(f_ptr(a, a.fkp, a.fbu, a.fbr, a.ftv, jj, kind_e, idx) + q);
    } else {
      tt[i] = 0.0;
      d[i] = czero();
    }
  }
#pragma unroll
  for (int lev = 1; lev < QM + 2; ++lev) {
#pragma unroll
    for (int i = 0; i + lev < QM + 2; ++i)
      if (i + lev < j.npts) d[i] = (1.0 / (tt[i + lev] - tt[i])) * (d[i + 1] - d[i]);
  }
  return j.coef * d[0];
}

__global__ void __launch_bounds__(256) ad_norm(PA a, AA b, int n, int nj, NormJob j0, NormJob j1,
                                               uint32_t seq) {
  const int64_t E = E_(a);
  const int64_t tot = (int64_t)nelem(a, n) * E;
  __shared__ double red[2][256];
  __shared__ bool last;
  double acc[2] = {0.0, 0.0};
  for (int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x; gid < tot;
       gid += (int64_t)gridDim.x * 256) {
    const int e = (int)(gid / E), q = (int)(gid % E);
    int kind_e, idx;
    elem_of(a, n, e, kind_e, idx);
    const kbe_c128 *pp = prev_ptr(a, a.kp, a.tv, n, kind_e, idx);
    const int r = q / a.N, c = q % a.N;
    const cd prev = pp ? ld(pp + q) : cd{0.0, r == c ? -1.0 : 0.0};
    const double wt = 1.0 / (b.rtol * sqrt(prev.re * prev.re + prev.im * prev.im) + b.atol);
    for (int jj = 0; jj < nj; ++jj) {
      const cd v = norm_term(a, b, n, e, q, kind_e, idx, gid, jj == 0 ? j0 : j1);
      const double m = sqrt(v.re * v.re + v.im * v.im) * wt;
      acc[jj] += m * m;
    }
  }
  const int tid = threadIdx.x;
  red[0][tid] = acc[0];
  red[1][tid] = acc[1];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      red[0][tid] += red[0][tid + off];
      red[1][tid] += red[1][tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    b.part[blockIdx.x] = red[0][0];
    b.part[NPART + blockIdx.x] = red[1][0];
    __threadfence();
    last = atomicAdd(b.done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  for (int jj = 0; jj < nj; ++jj) {
    double sum = 0.0;
    for (int i = tid; i < (int)gridDim.x; i += 256) sum += b.part[jj * NPART + i];
    red[0][tid] = sum;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (tid < off) red[0][tid] += red[0][tid + off];
      __syncthreads();
    }
    if (tid == 0) b.res[jj] = sqrt(red[0][0] / (double)(tot > 0 ? tot : 1));
    __syncthreads();
  }
  if (tid == 0) {
    *b.done = 0u;
    __threadfence_system();  // the norms reach host memory before the sequence number
    *b.flag = seq;
  }
}

// Keep the Sigma row and eps of the accepted step n (the history of later reconstructions).
__global__ void ad_keep(PA a, AA b, int n) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nrow = (int64_t)(n + 1) * E;
  if (gid < nrow) {
    st(b.Sret + (int64_t)n * a.nt * E + gid, ld(b.sret + gid));
    st(b.Sles + (int64_t)n * a.nt * E + gid, ld(b.sles + gid));
  } else if (gid < nrow + (int64_t)a.ntau * E) {
    const int64_t g2 = gid - nrow;
    st(b.Stv + (int64_t)n * a.ntau * E + g2, ld(b.stv + g2));
  } else if (gid < nrow + (int64_t)a.ntau * E + E) {
    const int64_t g3 = gid - nrow - (int64_t)a.ntau * E;
    st(b.epsall + (int64_t)n * E + g3, ld(a.eps + g3));
  }
}

// History sums of Eq. KBE2 at row j < n and column n (the lesser form C^< and the greater form
// C^>), for j = j0..n-1: I^R with upper limit t_j (weights row j), I^< with upper limit t_n
// (weights row n), Sigma(t_j, t_s) for s > j read from row s through the symmetry
// Sigma(t_j,t_s) = -Sigma(t_s,t_j)^dagger (Sigma^> = Sigma^R + Sigma^< in the stored rows).
// Upper history sums of step n at rows j0 <= j < n, in two stages.  Stage one: block (c, j - j0)
// takes terms u in [c UCH, (c + 1) UCH) of row j's three sums, numbered
//   u <  j + 1                      : w_j[s] Sigma^R(t_j,t_s) G^{<,>}(t_s,t_n), s = u;
//   u <  j + n + 2                  : w_n[s] Sigma^{<,>}(t_j,t_s) G^A(t_s,t_n), s = u - j - 1;
//   u <  j + n + 2 + ntau           : -i wtau[l] Sigma^](t_j,tau_l) G^[(tau_l,t_n), l = u - j - n - 2;
// each thread one element of the block for every lanes-th term (the term's blocks staged in LDS
// by its lane group, one element per thread), the lanes summed in LDS in a fixed order, and
// writes its chunk's partial sums of C^< (ret + les + mixed) and C^> (the same with G^>,
// Sigma^>).  Stage two sums the chunks in order.  The result does not depend on the
// launch beyond the rounding of the fixed summation order.
constexpr int UCH = 64;
static_assert(KBE_NMAX * KBE_NMAX <= 256, "ad_upper_part: one block element per thread");

__host__ __device__ __forceinline__ int upper_terms(int j, int n, int ntau) { return j + n + 2 + ntau; }

__global__ void __launch_bounds__(256) ad_upper_part(PA a, AA b, int n, int j0) {
  const int64_t E = E_(a);  // <= 256 (N <= KBE_NMAX)
  const int N = a.N;
  const int jj = blockIdx.y, j = j0 + jj, chunk = blockIdx.x, tid = threadIdx.x;
  const int lanes = 256 / (int)E;
  const int lane = tid / (int)E, q = tid % (int)E, r = q / N, c = q % N;
  const bool act = lane < lanes;
  const int u0 = chunk * UCH, uend = min(u0 + UCH, upper_terms(j, n, a.ntau));
  const double *wj = b.w + (int64_t)j * a.nt, *wn = b.w + (int64_t)n * a.nt;
  const int J = a.ntau - 1;
  // the blocks of each lane group's current term, staged element by element (coalesced) and
  // then read from LDS by the group's threads
  __shared__ cd blk[3][256];
  __shared__ cd red[2][256];
  cd cl = czero(), cg = czero();
  const int iters = (UCH + lanes - 1) / lanes;
  for (int it = 0; it < iters; ++it) {
    const int u = u0 + lane + it * lanes;
    const bool has = act && u < uend;
    if (has) {
      const kbe_c128 *P0, *P1, *P2 = nullptr;
      if (u <= j) {  // Sigma^R(t_j,t_s), G^<(s,n) = kp[s][n], G^R(n,s) = kp[n][s]
        const int s = u;
        P0 = b.Sret + ((int64_t)j * a.nt + s) * E;
        P1 = a.kp + ((int64_t)s * a.ldt + n) * E;
        P2 = a.kp + ((int64_t)n * a.ldt + s) * E;
      } else if (u <= j + n + 1) {  // Sigma^<, Sigma^R at (t_j,t_s) or (t_s,t_j); G^R(n,s)
        const int s = u - j - 1;
        const int64_t row = s <= j ? (int64_t)j * a.nt + s : (int64_t)s * a.nt + j;
        P0 = b.Sles + row * E;
        P1 = b.Sret + row * E;
        P2 = s < n ? a.kp + ((int64_t)n * a.ldt + s) * E : a.rdiag + n * E;
      } else {  // Sigma^](t_j,tau_l), G^](t_n,tau_{J-l})
        const int l = u - j - n - 2;
        P0 = b.Stv + ((int64_t)j * a.ntau + l) * E;
        P1 = a.tv + ((int64_t)n * a.ntau + (J - l)) * E;
      }
      blk[0][tid] = ld(P0 + q);
      blk[1][tid] = ld(P1 + q);
      if (P2) blk[2][tid] = ld(P2 + q);
    }
    __syncthreads();
    if (has) {
      const cd *B0 = blk[0] + lane * E, *B1 = blk[1] + lane * E, *B2 = blk[2] + lane * E;
      if (u <= j) {
        const int s = u;
        cd x = czero(), y = czero();
        for (int k = 0; k < N; ++k) {
          const cd sr = B0[r * N + k];
          const cd gl = B1[k * N + c];
          const cd gg = gl - cj(B2[c * N + k]);  // G^>(s,n) = kp[s][n] - kp[n][s]^dagger
          x = x + sr * gl;
          y = y + sr * gg;
        }
        cl = cl + wj[s] * x;
        cg = cg + wj[s] * y;
      } else if (u <= j + n + 1) {
        const int s = u - j - 1;
        cd x = czero(), y = czero();
        for (int k = 0; k < N; ++k) {
          cd sl, sg;
          if (s <= j) {
            sl = B0[r * N + k];
            sg = sl + B1[r * N + k];
          } else {
            const cd l = B0[k * N + r];
            const cd g = l + B1[k * N + r];
            sl = -cj(l);
            sg = -cj(g);
          }
          const cd ga = cj(B2[c * N + k]);  // G^A(s,n)[k][c] = conj(G^R(n,s)[c][k])
          x = x + sl * ga;
          y = y + sg * ga;
        }
        cl = cl + wn[s] * x;
        cg = cg + wn[s] * y;
      } else {
        const int l = u - j - n - 2;
        cd x = czero();
        for (int k = 0; k < N; ++k) x = x + B0[r * N + k] * cj(B1[c * N + k]);
        x = mul_mi(a.wtau_[l] * x);
        cl = cl + x;
        cg = cg + x;
      }
    }
    __syncthreads();
  }
  kbe_c128 *out = b.upart + (((int64_t)chunk * QM + jj) * 2) * E;
  red[0][tid] = cl;
  red[1][tid] = cg;
  __syncthreads();
  if (tid < E) {
    cd sl = red[0][tid], sg = red[1][tid];
    for (int i = 1; i < lanes; ++i) {
      sl = sl + red[0][i * E + tid];
      sg = sg + red[1][i * E + tid];
    }
    st(out + tid, sl);
    st(out + E + tid, sg);
  }
}

__global__ void ad_upper_sum(PA a, AA b, int n, int j0, int nchunk) {
  const int64_t E = E_(a);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)(n - j0) * E) return;
  const int jj = (int)(gid / E), q = (int)(gid % E);
  const int nc = (upper_terms(j0 + jj, n, a.ntau) + UCH - 1) / UCH;  // chunks of row j (<= nchunk)
  cd cl = czero(), cg = czero();
  for (int c = 0; c < nc && c < nchunk; ++c) {
    const kbe_c128 *in = b.upart + (((int64_t)c * QM + jj) * 2) * E;
    cl = cl + ld(in + q);
    cg = cg + ld(in + E + q);
  }
  st(b.Cl + (int64_t)jj * E + q, cl);
  st(b.Cg + (int64_t)jj * E + q, cg);
}

// Right sides of the blocks born at t_n below their birth: U_n at t_j, i (G^<(t_n,t_j) eps_j -
// C^<(j,n)^dagger) with G^<(t_n,t_j) = -kp[j][n]^dagger; R_n (continued: -kp[n][j]^dagger) at
// t_j, -i (eps_j (-kp[n][j]^dagger) + C^>(j,n) - C^<(j,n)).
__global__ void ad_recon(PA a, AA b, int n, int j0) {
  const int64_t E = E_(a);
  const int N = a.N;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)(n - j0) * E) return;
  const int jj = (int)(gid / E), j = j0 + jj, q = (int)(gid % E), r = q / N, c = q % N;
  const kbe_c128 *ep = b.epsall + (int64_t)j * E;
  const kbe_c128 *U = a.kp + ((int64_t)j * a.ldt + n) * E;   // kp[j][n]
  const kbe_c128 *R = a.kp + ((int64_t)n * a.ldt + j) * E;   // kp[n][j]
  const kbe_c128 *Cl = b.Cl + (int64_t)jj * E, *Cg = b.Cg + (int64_t)jj * E;
  cd fu = czero(), fr = czero();
  for (int k = 0; k < N; ++k) {
    fu = fu - cj(ld(U + k * N + r)) * ld(ep + k * N + c);  // (-kp[j][n]^dagger) eps_j
    fr = fr - ld(ep + r * N + k) * cj(ld(R + c * N + k));  // eps_j (-kp[n][j]^dagger)
  }
  fu = mul_i(fu - cj(ld(Cl + c * N + r)));
  fr = mul_mi(fr + ld(Cg + q) - ld(Cl + q));
  const int i = n - 1 - j;  // < QM
  st(a.fpu + ((int64_t)n * QM + i) * E + q, fu);
  st(a.fpr + ((int64_t)n * QM + i) * E + q, fr);
}

}  // namespace

size_t prop_ws_bytes(int N, int nt, int ntau, int64_t ldt, int K) {
  return layout(N, nt, ntau, ldt, K).total;
}

hipError_t launch_propagate(const kbe_prop *P, const kbe_wts *W, const kbe_green *G,
                            double *dens, void *ws, hipStream_t st) {
  Ctx x = make_ctx(P, W, G, ws, st);
  PA &a = x.a;
  const int64_t E = (int64_t)a.N * a.N;
  hipLaunchKernelGGL(prop_init, dim3(blocks((int64_t)(a.nt + a.ntau) * E)), dim3(256), 0, st, a);
  hipError_t e = evaluate(x, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prop_rhs, dim3(blocks((int64_t)(a.ntau + 3) * E)), dim3(256), 0, st, a, 0, 1);
  hipLaunchKernelGGL(prop_dens, dim3(1), dim3(64), 0, st, a, 0, dens);
  for (int n = 1; n < a.nt; ++n) {
    const int64_t ne = 2 * n + 1 + a.ntau;
    hipLaunchKernelGGL(prop_predict, dim3(blocks(ne * E)), dim3(256), 0, st, a, n);
    for (int it = 1; it <= a.K; ++it) {
      if ((e = evaluate(x, n)) != hipSuccess) return e;
      hipLaunchKernelGGL(prop_rhs, dim3(blocks(ne * E)), dim3(256), 0, st, a, n, 0);
      hipLaunchKernelGGL(prop_commit, dim3(blocks(ne * E)), dim3(256), 0, st, a, n, it);
    }
    if ((e = evaluate(x, n)) != hipSuccess) return e;
    hipLaunchKernelGGL(prop_rhs, dim3(blocks((ne + 2) * E)), dim3(256), 0, st, a, n, 1);
    hipLaunchKernelGGL(prop_dens, dim3(1), dim3(64), 0, st, a, n, dens);
  }
  return hipGetLastError();
}

namespace {

// Host-side helpers of the adaptive controller (the same formulas as the oracle's).
double poly_integral(const double *x, int k, double a, double b) {  // int_a^b prod (s - x_i) ds
  // Gauss-Legendre with m >= (k + 1) / 2 points (Newton on the three-term recurrence)
  const int m = k / 2 + 2;
  double acc = 0.0;
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
    const double wgt = 2.0 / ((1.0 - z * z) * dp * dp);
    const double sv = 0.5 * (b - a) * z + 0.5 * (a + b);
    double pr = 1.0;
    for (int l = 0; l < k; ++l) pr *= sv - x[l];
    acc += wgt * pr;
  }
  return 0.5 * (b - a) * acc;
}

double factorial(int q) {
  double f = 1.0;
  for (int i = 2; i <= q; ++i) f *= i;
  return f;
}

// Term chunks of the upper history sums at the last step of a grid of nt points.
int upper_chunks(int nt, int ntau) { return (2 * nt + ntau + UCH - 1) / UCH; }

struct ALay {
  size_t fkp, fbu, fbr, ftv, fpu, fpr, t, w, eps, sret, sles, stv, Sret, Sles, Stv, epsall, IRl,
      ILl, Itv, Jtv, IRg, ILg, base, ynext, ypred, ubuf, Cl, Cg, upart, amt, abt, part, done, kbuf,
      cws, total;
};

ALay alayout(int N, int nt, int ntau) {
  const size_t E = (size_t)N * N * sizeof(kbe_c128);
  const size_t nt2 = (size_t)nt * nt, ne = (size_t)(2 * nt + 1 + ntau + 2);
  ALay L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t r = o; o += al(bytes); return r; };
  L.fkp = take(nt2 * E);
  L.fbu = take(nt * E);
  L.fbr = take(nt * E);
  L.ftv = take((size_t)nt * ntau * E);
  L.fpu = take((size_t)nt * QM * E);
  L.fpr = take((size_t)nt * QM * E);
  L.t = take(nt * sizeof(double));
  L.w = take(nt2 * sizeof(double));
  L.eps = take(E);
  L.sret = take(nt * E);
  L.sles = take(nt * E);
  L.stv = take(ntau * E);
  L.Sret = take(nt2 * E);
  L.Sles = take(nt2 * E);
  L.Stv = take((size_t)nt * ntau * E);
  L.epsall = take(nt * E);
  L.IRl = take(nt * E);
  L.ILl = take(nt * E);
  L.Itv = take(nt * E);
  L.Jtv = take(ntau * E);
  L.IRg = take(nt * E);
  L.ILg = take(nt * E);
  L.base = take(ne * E);
  L.ynext = take(ne * E);
  L.ypred = take(ne * E);
  L.ubuf = take((size_t)KM * E);
  L.Cl = take((size_t)QM * E);
  L.Cg = take((size_t)QM * E);
  L.upart = take((size_t)upper_chunks(nt, ntau) * QM * 2 * E);
  L.amt = take(KM * KM * sizeof(double));
  L.abt = take(KM * KM * sizeof(double));
  L.part = take(2 * NPART * sizeof(double));
  L.done = take(2 * sizeof(uint32_t));
  L.kbuf = take((size_t)nt * KSW * sizeof(int32_t));
  const int n = nt - 1;
  L.cws = take(collision_ws_bytes_rows(N, nt, ntau, KBE_OUT_ALL | KBE_INT_BOTH));
  L.total = o;
  return L;
}

}  // namespace

size_t prop_adaptive_ws_bytes(int N, int nt, int ntau) { return alayout(N, nt, ntau).total; }

// Page-locked, coherent host memory for the norms the controller reads, held for one call:
// res[0..1] and, at byte 64, the sequence number of the last norm launch that wrote them.
struct HostRes {
  char *host = nullptr, *dev = nullptr;
  hipError_t alloc() {
    hipError_t e = hipHostMalloc((void **)&host, 4096,
                                 hipHostMallocMapped | hipHostMallocPortable |
                                     hipHostMallocCoherent);
    if (e != hipSuccess) {
      host = nullptr;
      return e;
    }
    std::memset(host, 0, 4096);
    return hipHostGetDevicePointer((void **)&dev, host, 0);
  }
  const volatile double *res() const { return (const volatile double *)host; }
  const volatile uint32_t *flag() const { return (const volatile uint32_t *)(host + 64); }
  ~HostRes() {
    if (host) (void)hipHostFree(host);
  }
};

hipError_t launch_propagate_adaptive(const kbe_prop *P, const kbe_adapt_ctl *ctl,
                                     const kbe_wts *W, const kbe_green *G, double *dens,
                                     kbe_adapt_trace *tr, void *ws, hipStream_t st,
                                     int *stalled) {
  *stalled = 0;
  const ALay L = alayout(G->N, G->nt, G->ntau);
  char *wsb = (char *)ws;
  auto c = [&](size_t off) { return (kbe_c128 *)(wsb + off); };
  PA a{};
  a.N = G->N;
  a.nt = G->nt;
  a.ntau = G->ntau;
  a.K = 0;
  a.ldt = G->ldt;
  a.kp = G->kp;
  a.rdiag = G->rdiag;
  a.tv = G->tv;
  a.mat = G->mat;
  a.h0 = P->h0;
  a.u = P->u;
  a.amp = P->pulse_amp;
  a.t0 = P->pulse_t0;
  a.sig = P->pulse_sigma;
  a.fkp = c(L.fkp);
  a.fbu = c(L.fbu);
  a.fbr = c(L.fbr);
  a.ftv = c(L.ftv);
  a.fpu = c(L.fpu);
  a.fpr = c(L.fpr);
  a.eps = c(L.eps);
  a.IRl = c(L.IRl);
  a.ILl = c(L.ILl);
  a.Itv = c(L.Itv);
  a.Jtv = c(L.Jtv);
  a.IRg = c(L.IRg);
  a.ILg = c(L.ILg);
  a.base = c(L.base);
  a.ynext = c(L.ynext);
  a.adaptive = 1;
  a.q = 1;
  a.amt = (const double *)(wsb + L.amt);
  a.abt = (const double *)(wsb + L.abt);
  a.wtau_ = W->wtau;
  double *tdev = (double *)(wsb + L.t);
  double *wdev = (double *)(wsb + L.w);
  a.t = tdev;
  AA b{};
  b.t = tdev;
  b.w = wdev;
  b.ypred = c(L.ypred);
  b.sret = c(L.sret);
  b.sles = c(L.sles);
  b.stv = c(L.stv);
  b.Sret = c(L.Sret);
  b.Sles = c(L.Sles);
  b.Stv = c(L.Stv);
  b.epsall = c(L.epsall);
  b.ubuf = c(L.ubuf);
  b.Cl = c(L.Cl);
  b.Cg = c(L.Cg);
  b.upart = c(L.upart);
  b.part = (double *)(wsb + L.part);
  b.done = (uint32_t *)(wsb + L.done);
  b.cdone = b.done + 1;
  b.kbuf = (int32_t *)(wsb + L.kbuf);
  // the norms the controller reads: written by the kernels into page-locked host memory, read
  // after the stream is synchronised (no copy operations)
  HostRes hres;
  hipError_t e = hres.alloc();
  if (e != hipSuccess) return e;
  b.res = (double *)hres.dev;
  b.flag = (volatile uint32_t *)(hres.dev + 64);
  uint32_t seq = 0;
  b.rtol = ctl->rtol;
  b.atol = ctl->atol;
  const int N = a.N, nt = a.nt, ntau = a.ntau;
  const int64_t E = (int64_t)N * N;
  kbe_green Gc = *G;
  kbe_sigma_row sig{b.sret, b.sles, ntau ? b.stv : nullptr};
  const bool th = ntau > 0;
  // history weights: the collision reads rows 0..n of w (row stride nt)
  kbe_wts Wc{wdev, W->wtau, W->wtau_fwd};
  auto coll = [&](int n) -> hipError_t {
    Params p{};
    p.N = N;
    p.nt = nt;
    p.ntau = ntau;
    p.J = ntau - 1;
    p.n = n;
    p.m0 = 0;
    p.m1 = n + 1;
    p.ldt = a.ldt;
    p.kp = a.kp;
    p.rdiag = a.rdiag;
    p.tv = a.tv;
    p.mat = a.mat;
    p.ret = sig.ret;
    p.les = sig.les;
    p.stv = sig.tv;
    p.w = Wc.w;
    p.wtau = Wc.wtau;
    p.wf = Wc.wtau_fwd;
    set_flags(p, FL, th);
    return launch_collision_both(p, a.IRl, a.ILl, a.Itv, a.Jtv, a.IRg, a.ILg, wsb + L.cws, st);
  };
  // one evaluation of the right sides at the current values of step n; kslot: which evaluation
  // of the step it is (where its history order is recorded, n >= 1)
  auto evaluate = [&](int n, int kslot) -> hipError_t {
    hipError_t r = launch_sigma_row(&Gc, a.u, n, &sig, st);
    if (r != hipSuccess) return r;
    if (n >= 1) {
      const int K = ctl->kmax < n + 1 ? ctl->kmax : n + 1;
      hipLaunchKernelGGL(ad_choose, dim3(blocks((int64_t)K * E)), dim3(256), 0, st, a, b, n, K,
                         (int64_t)n * KSW + kslot);
    }
    if ((r = coll(n)) != hipSuccess) return r;
    hipLaunchKernelGGL(prop_eps, dim3(1), dim3(256), 0, st, a, n);
    return hipGetLastError();
  };
  hipError_t nerr = hipSuccess;
  // one or two norms (jobs) of step n: the host polls the launch's sequence number in host
  // memory; every 256 polls it asks whether the stream has finished or failed, so an error or a
  // launch that wrote nothing ends the wait
  auto launch_norms = [&](int n, int nj, NormJob j0, NormJob j1) {
    const int64_t tot = (int64_t)(2 * n + 1 + ntau) * E;
    int nb = (int)((tot + 255) / 256);
    nb = nb < NPART ? nb : NPART;
    ++seq;
    hipLaunchKernelGGL(ad_norm, dim3(nb), dim3(256), 0, st, a, b, n, nj, j0, j1, seq);
    const hipError_t r = hipGetLastError();
    if (r != hipSuccess) nerr = r;
  };
  auto wait_norms = [&](int nj, double *out) {
    hipError_t r = nerr;
    for (uint64_t spin = 1; r == hipSuccess; ++spin) {
      if (*hres.flag() == seq) break;
      if ((spin & 255) == 0) {
        const hipError_t qs = hipStreamQuery(st);
        if (qs == hipErrorNotReady) continue;
        if (qs != hipSuccess) r = qs;
        else if (*hres.flag() != seq) r = hipErrorUnknown;  // the stream is idle: never written
        break;
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    for (int j = 0; j < nj; ++j) out[j] = r == hipSuccess ? hres.res()[j] : NAN;
    if (r != hipSuccess) nerr = r;
  };
  // the history orders of steps 1..n-1 into the trace (slots beyond a step's evaluations zero)
  auto finish = [&](int n) -> hipError_t {
    tr->nt = n;
    std::vector<int32_t> ks((size_t)n * KSW);
    hipError_t r = hipMemcpyAsync(ks.data(), b.kbuf, ks.size() * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, st);
    if (r == hipSuccess) r = hipStreamSynchronize(st);
    if (r != hipSuccess) return r;
    for (int j = 1; j < n; ++j)
      for (int i = 0; i < KSW; ++i)
        tr->ks[(int64_t)j * KSW + i] = i <= tr->m[j] ? ks[(size_t)j * KSW + i] : 0;
    return hipSuccess;
  };
  std::vector<double> t(1, 0.0);
  // t = 0: the initial state, its right sides, the weights row 0 (zero)
  hipLaunchKernelGGL(fill_zero<double>, dim3(blocks((int64_t)nt * nt)), dim3(256), 0, st, wdev,
                     (int64_t)nt * nt);
  hipLaunchKernelGGL(ad_set_t, dim3(1), dim3(64), 0, st, tdev, 0, 0.0);
  hipLaunchKernelGGL(fill_zero<uint32_t>, dim3(1), dim3(64), 0, st, b.done, (int64_t)2);
  hipLaunchKernelGGL(prop_init, dim3(blocks((int64_t)(nt + ntau) * E)), dim3(256), 0, st, a);
  if ((e = evaluate(0, 0)) != hipSuccess) return e;
  hipLaunchKernelGGL(prop_rhs, dim3(blocks((int64_t)(ntau + 3) * E)), dim3(256), 0, st, a, 0, 1);
  hipLaunchKernelGGL(ad_keep, dim3(blocks((int64_t)(1 + ntau + 1) * E)), dim3(256), 0, st, a, b, 0);
  hipLaunchKernelGGL(prop_dens, dim3(1), dim3(64), 0, st, a, 0, dens);
  tr->t[0] = 0.0;
  tr->q[0] = 0;
  tr->m[0] = 0;
  tr->err[0] = 0.0;
  for (int i = 0; i < KSW; ++i) tr->ks[i] = 0;
  tr->rejected = 0;
  double h = ctl->h0;
  int q = 1, at_q = 0, n = 1;
  while (n < nt && t.back() < ctl->t_end * (1.0 - 1e-14)) {
    int nfail = 0, m = 0;
    double E_err = 0.0, tn = 0.0;
    for (;;) {
      h = h < ctl->t_end - t.back() ? h : ctl->t_end - t.back();
      if (!(h > 1e-13 * (t.back() > 1.0 ? t.back() : 1.0))) {  // step size underflow
        *stalled = 1;
        if ((e = finish(n)) != hipSuccess) return e;
        return hipGetLastError();
      }
      q = q < n ? q : n;
      tn = t.back() + h;
      const int kam = (ctl->kmax > q ? ctl->kmax : q);  // the rules store t_n in t[n] too
      if ((e = launch_interval_weights(tdev, n, tn, kam, q, (double *)(wsb + L.amt),
                                       (double *)(wsb + L.abt), st)) != hipSuccess)
        return e;
      a.q = q;
      // error-estimate coefficient (Milne's device, the same formula as the oracle's)
      std::vector<double> tg(t);
      tg.push_back(tn);
      const double cam = poly_integral(&tg[n - q + 1], q, tg[n - 1], tg[n]) / factorial(q);
      const double cab = poly_integral(&tg[n - q], q, tg[n - 1], tg[n]) / factorial(q);
      const double C = fabs(cam / (cab - cam));
      const int64_t ne = 2 * n + 1 + ntau;
      hipLaunchKernelGGL(ad_predict, dim3(blocks(ne * E)), dim3(256), 0, st, a, b, n);
      bool conv = false;
      double R = 1.0, dprev = 0.0;
      m = 0;
      if ((e = evaluate(n, 0)) != hipSuccess) return e;
      while (m < ctl->maxcor) {
        ++m;
        hipLaunchKernelGGL(prop_rhs, dim3(blocks(ne * E)), dim3(256), 0, st, a, n, 0);
        // the correction's norm, and the local error should this iterate be the last one
        launch_norms(n, 2, NormJob{0, 0, 0.0, 0.0}, NormJob{3, 0, C, 0.0});
        hipLaunchKernelGGL(prop_commit, dim3(blocks(ne * E)), dim3(256), 0, st, a, n, -1);
        // queued before the decision is known: the next iteration's evaluation and the final
        // evaluation at the accepted values are the same computation on the committed iterate
        // (it is only wasted when the step is rejected)
        if ((e = evaluate(n, m)) != hipSuccess) return e;
        double dv[2];
        wait_norms(2, dv);
        if (nerr != hipSuccess) return nerr;
        const double d = dv[0];
        E_err = dv[1];
        if (!std::isfinite(d)) break;  // a non-finite iterate: not converged
        if (m > 1) R = dprev > 0 ? (0.3 * R > d / dprev ? 0.3 * R : d / dprev) : 0.0;
        if ((R < 1.0 ? R : 1.0) * d * C < 0.1) {
          conv = true;
          break;
        }
        if (m > 1 && d > 2.0 * dprev) break;
        dprev = d;
      }
      if (!conv || !std::isfinite(E_err)) {
        ++tr->rejected;
        h *= 0.25;
        continue;
      }
      if (E_err > 1.0) {
        ++tr->rejected;
        ++nfail;
        if (nfail >= 3) {
          q = 1;
          at_q = 0;
          h *= 0.25;
        } else {
          const double eta = 0.9 * pow(E_err, -1.0 / (q + 1));
          h *= eta > 0.9 ? 0.9 : (eta < 0.2 ? 0.2 : eta);
        }
        continue;
      }
      break;
    }
    // accept: the right sides at the accepted values (evaluated above), the step's history
    const int64_t ne = 2 * n + 1 + ntau;
    hipLaunchKernelGGL(prop_rhs, dim3(blocks((ne + 2) * E)), dim3(256), 0, st, a, n, 1);
    t.push_back(tn);
    tr->t[n] = tn;
    tr->q[n] = q;
    tr->m[n] = m;
    tr->err[n] = E_err;
    // the error estimates at orders q - 1 and q + 1 (once q + 1 steps were taken at order q), in
    // one launch ahead of the rest of the step's kernels; read before the next step
    ++at_q;
    NormJob jb[2];
    int dqs[2], nj = 0;
    if (at_q >= q + 1) {
      for (int dq = -1; dq <= 1; dq += 2) {
        const int qq = q + dq, npts = qq + 1;
        if (qq < 1 || qq > ctl->qmax || npts > n + 1) continue;
        jb[nj] = NormJob{2, npts, 0.0, poly_integral(&t[n - qq + 1], qq, t[n - 1], t[n])};
        dqs[nj++] = dq;
      }
      if (nj > 0) launch_norms(n, nj, jb[0], nj > 1 ? jb[1] : NormJob{});
    }
    hipLaunchKernelGGL(ad_keep, dim3(blocks((int64_t)(n + 1 + ntau + 1) * E)), dim3(256), 0, st, a,
                       b, n);
    hipLaunchKernelGGL(prop_dens, dim3(1), dim3(64), 0, st, a, n, dens);
    const int j0 = n - ctl->qmax > 0 ? n - ctl->qmax : 0;
    const int nch = (upper_terms(n - 1, n, ntau) + UCH - 1) / UCH;
    hipLaunchKernelGGL(ad_upper_part, dim3(nch, n - j0), dim3(256), 0, st, a, b, n, j0);
    hipLaunchKernelGGL(ad_upper_sum, dim3(blocks((int64_t)(n - j0) * E)), dim3(256), 0, st, a, b,
                       n, j0, nch);
    hipLaunchKernelGGL(ad_recon, dim3(blocks((int64_t)(n - j0) * E)), dim3(256), 0, st, a, b, n,
                       j0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // next step size and order
    double eta = 1.0 / (pow(6.0 * E_err, 1.0 / (q + 1)) + 1e-6);
    int qn = q;
    if (nj > 0) {
      double Eq[2];
      wait_norms(nj, Eq);
      if (nerr != hipSuccess) return nerr;
      for (int j = 0; j < nj; ++j) {
        if (!std::isfinite(Eq[j])) continue;
        const int qq = q + dqs[j];
        const double bias = dqs[j] < 0 ? 6.0 : 10.0;
        const double e2 = 1.0 / (pow(bias * Eq[j], 1.0 / (qq + 1)) + 1e-6);
        if (e2 > eta) {
          eta = e2;
          qn = qq;
        }
      }
    }
    if (eta >= 1.5) {
      if (qn != q) at_q = 0;
      q = qn;
      h *= eta < 10.0 ? eta : 10.0;
    }
    ++n;
  }
  if ((e = finish(n)) != hipSuccess) return e;
  if (t.back() < ctl->t_end * (1.0 - 1e-14)) *stalled = 2;  // capacity exhausted
  return hipGetLastError();
}

hipError_t launch_propagate_vjp(const kbe_prop *P, const kbe_wts *W, const kbe_green *G,
                                const double *gdens, double *gu, double *gamp, void *ws,
                                hipStream_t st) {
  Ctx x = make_ctx(P, W, G, ws, st);
  PA &a = x.a;
  const int64_t E = (int64_t)a.N * a.N;
  const Layout &L = x.L;
  // zero the gradient arrays (fill kernels: no memset nodes if the caller captures the call)
  const size_t zb = L.gfkp - L.gkp, zf = L.ybar - L.gfkp;
  hipLaunchKernelGGL(fill_zero<double>, dim3(blocks((int64_t)(zb / 8))), dim3(256), 0, st,
                     (double *)(x.ws + L.gkp), (int64_t)(zb / 8));
  hipLaunchKernelGGL(fill_zero<double>, dim3(blocks((int64_t)(zf / 8))), dim3(256), 0, st,
                     (double *)(x.ws + L.gfkp), (int64_t)(zf / 8));
  hipLaunchKernelGGL(fill_zero<double>, dim3(1), dim3(64), 0, st, gu, (int64_t)a.N);
  hipLaunchKernelGGL(fill_zero<double>, dim3(1), dim3(64), 0, st, gamp, (int64_t)1);
  hipLaunchKernelGGL(prop_seed, dim3(blocks((int64_t)a.nt * a.N)), dim3(256), 0, st, a, gdens);
  hipError_t e;
  for (int n = a.nt - 1; n >= 1; --n) {
    const int64_t ne = 2 * n + 1 + a.ntau;
    // the final evaluation (row/column n holds the accepted values)
    hipLaunchKernelGGL(prop_gather_final, dim3(blocks((ne + 2) * E)), dim3(256), 0, st, a, n);
    if ((e = evaluate_vjp(x, n, 1, gu, gamp)) != hipSuccess) return e;
    for (int it = a.K; it >= 1; --it) {
      hipLaunchKernelGGL(prop_take, dim3(blocks(ne * E)), dim3(256), 0, st, a, n, it == a.K);
      hipLaunchKernelGGL(prop_restore, dim3(blocks(ne * E)), dim3(256), 0, st, a, n, it - 1);
      if ((e = evaluate_vjp(x, n, 0, gu, gamp)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(prop_predict_vjp, dim3(blocks(ne * E)), dim3(256), 0, st, a, n);
    hipLaunchKernelGGL(prop_restore, dim3(blocks(ne * E)), dim3(256), 0, st, a, n, a.K);
  }
  hipLaunchKernelGGL(prop_gather_final, dim3(blocks((int64_t)(a.ntau + 3) * E)), dim3(256), 0, st,
                     a, 0);
  if ((e = evaluate_vjp(x, 0, 1, gu, gamp)) != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace kbe
