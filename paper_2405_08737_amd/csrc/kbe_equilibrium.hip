// Interacting equilibrium initial state: the Matsubara Dyson equation of the local-U second-Born
// approximation on the uniform tau grid tau_j = j beta / J (ntau = J + 1 points, tau_0 = 0+,
// tau_J = beta-).
//
// The propagations take G^M as their initial condition (Sec. "Kadanoff Baym Equations"); a
// G^M that is an equilibrium of the interacting system is what makes the unperturbed
// propagation stationary.  In equilibrium Eq. KBE3 at t = 0, with the boundary conditions of
// Eq. BC, reduces to  -dG^M/dtau = eps G^M + int_0^beta Sigma^M(u) G^M(tau - u) du
// (antiperiodic in tau), whose integral form is the Dyson equation G^M = G0 + G0 * Sigma^M * G^M
// with G0 the free Matsubara function of eps.  Per iteration:
//   eps   = h0 + diag(u_i n_i) - mu, n_i = -G^M_ii(beta-)       (Hartree term of Eq. eps)
//   G0    = -V exp(-e tau) (1 - f(e)) V^T                        (eigendecomposition of eps)
//   S     = Sigma^M_ij(tau) = u_i u_j G_ij(tau)^2 G_ji(beta - tau)  (Eq. SE at t = 0)
//   X     = S * G,  Gn = G0 + G0 * X,  G <- (1 - mix) G + mix Gn
// where (A * B)(tau_j) = sum_{l<=j} wf[j][l] A(tau_{j-l}) B(tau_l)
//                      - sum_{l>=j} wb[j][l] A(tau_{J+j-l}) B(tau_l),
// the integral split at u = tau_j (where A(tau_j - u) jumps), the part above it continued
// antiperiodically, wf the forward tau rule of the propagation and wb[j][l] = wf[J-j][J-l] its
// reflection, the rule over [tau_j, beta] on the uniform grid.
//
// G^M is real for the real symmetric h0 of the propagations, so the iteration runs in real FP64
// and writes the complex output once at the end.  Kernels (one launch each per iteration):
//   eq_eig    one block: parallel (round-robin) Jacobi on eps, N/2 disjoint rotations per round,
//             from the previous iteration's eigenvectors
//   eq_free   a block per tau point: G0 from (e, V), and the self-energy of the iterate
//   eq_conv4  a block per tau point (N a multiple of 4; eq_conv otherwise), the l-sum split over
//             slices of the block, 4 x 4 register tiles, LDS reduction; the second convolution
//             also forms Gn, mixes in place and reduces the change
// The host reads the change (8 bytes) once per iteration to decide convergence.
#include "kbe_internal.h"

#include <cmath>
#include <cstring>

namespace kbe {
namespace {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int EQ_T = 256;          // threads per block (>= KBE_NMAX^2)
constexpr int EQ_SWEEPS = 40;      // Jacobi sweep limit (5-6 sweeps for N <= 16 in practice)
static_assert(KBE_NMAX * KBE_NMAX <= EQ_T, "one thread per matrix element");

__device__ __forceinline__ size_t el(int j, int a, int b, int N) {
  return ((size_t)j * N + a) * N + b;
}

// Eigendecomposition of eps (hartree != 0: with the Hartree shift of G[J]; else of h0 - mu).
// warm != 0: start from the eigenvectors V_out of the previous call, i.e. diagonalise V^T eps V
// (nearly diagonal once the densities settle) and accumulate the rotations onto V.
// Round-robin ordering: in round r player r pairs with M-1 and (r+k) mod (M-1) with
// (r-k) mod (M-1), k = 1..M/2-1 (M = N rounded up to even; a pair with the dummy player N is
// idle).  The rotation of pair (p < q) zeroes A[p][q]: theta = (A_qq - A_pp) / (2 A_pq),
// t = sign(theta) / (|theta| + sqrt(theta^2 + 1)), c = 1 / sqrt(t^2 + 1), s = t c, and with
// J_pp = J_qq = c, J_pq = s, J_qp = -s the update is A <- J^T A J, V <- V J.  The rotations of
// one round act on disjoint planes, so they are applied together.  Also clears the change
// accumulator of the iteration.
__global__ void __launch_bounds__(EQ_T) eq_eig(const double *h0, const double *u, double mu,
                                               const double *G, int J, int N, int hartree,
                                               int warm, double *e_out, double *V_out,
                                               unsigned long long *chg) {
  __shared__ double A[2][KBE_NMAX][KBE_NMAX + 1], V[2][KBE_NMAX][KBE_NMAX + 1];
  __shared__ double jd[KBE_NMAX + 1], jo[KBE_NMAX + 1];
  __shared__ int pt[KBE_NMAX + 1];
  __shared__ double wo[EQ_T / 64], wt[EQ_T / 64];
  __shared__ int done;
  const int tid = threadIdx.x;
  const bool act = tid < N * N;
  const int a = act ? tid / N : 0, b = act ? tid % N : 0;
  if (tid == 0) *chg = 0ull;
  if (act) {
    double x = 0.5 * (h0[a * N + b] + h0[b * N + a]);
    if (a == b) {
      if (hartree) x += u[a] * -G[el(J, a, a, N)];
      x -= mu;
    }
    A[warm ? 1 : 0][a][b] = x;
    V[0][a][b] = warm ? V_out[a * N + b] : (a == b ? 1.0 : 0.0);
  }
  __syncthreads();
  if (warm) {  // A[0] = V^T eps V, through V[1] = eps V
    if (act) {
      double t = 0.0;
      for (int k = 0; k < N; ++k) t += A[1][a][k] * V[0][k][b];
      V[1][a][b] = t;
    }
    __syncthreads();
    if (act) {
      double t = 0.0;
      for (int k = 0; k < N; ++k) t += V[0][k][a] * V[1][k][b];
      A[0][a][b] = t;
    }
    __syncthreads();
  }
  const int M = N + (N & 1);
  int cur = 0;
  for (int sweep = 0; sweep < EQ_SWEEPS; ++sweep) {
    // squared off-diagonal and total norms: wave sums, then the waves in order
    double vo = 0.0, vt = 0.0;
    if (act) {
      const double x = A[cur][a][b];
      vt = x * x;
      vo = a != b ? vt : 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) {
      vo += __shfl_down(vo, o);
      vt += __shfl_down(vt, o);
    }
    if ((tid & 63) == 0) {
      wo[tid >> 6] = vo;
      wt[tid >> 6] = vt;
    }
    __syncthreads();
    if (tid == 0) {
      double off = 0.0, tot = 0.0;
      for (int w = 0; w < EQ_T / 64; ++w) {
        off += wo[w];
        tot += wt[w];
      }
      done = !(off > 1e-30 * tot);  // off-diagonal Frobenius norm below 1e-15 of the whole
    }
    __syncthreads();
    if (done) break;
    for (int r = 0; r < M - 1; ++r) {
      if (tid < M / 2) {
        int p, q;
        if (tid == 0) {
          p = r;
          q = M - 1;
        } else {
          p = (r + tid) % (M - 1);
          q = (r - tid + M - 1) % (M - 1);
        }
        if (p > q) {
          const int w = p;
          p = q;
          q = w;
        }
        double c = 1.0, s = 0.0;
        if (q < N) {
          const double apq = A[cur][p][q];
          if (apq != 0.0) {
            const double th = (A[cur][q][q] - A[cur][p][p]) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        pt[p] = q;
        pt[q] = p;
        jd[p] = c;
        jd[q] = c;
        jo[p] = -s;  // J[q][p]
        jo[q] = s;   // J[p][q]
      }
      __syncthreads();
      if (act) {
        // A'[a][b] = sum over k in {a, pa}, l in {b, pb} of J[k][a] A[k][l] J[l][b]
        const int pa = pt[a], pb = pt[b];
        const double da = jd[a], oa = jo[a], db = jd[b], ob = jo[b];
        double x = da * db * A[cur][a][b];
        double y = V[cur][a][b] * db;
        if (pb < N) {
          x += da * ob * A[cur][a][pb];
          y += V[cur][a][pb] * ob;
        }
        if (pa < N) {
          x += oa * db * A[cur][pa][b];
          if (pb < N) x += oa * ob * A[cur][pa][pb];
        }
        A[cur ^ 1][a][b] = x;
        V[cur ^ 1][a][b] = y;
      }
      cur ^= 1;
      __syncthreads();
    }
  }
  if (act) {
    V_out[a * N + b] = V[cur][a][b];
    if (a == b) e_out[a] = A[cur][a][a];
  }
}

// G0(tau_j) = V diag(x(tau_j)) V^T, x_k = -exp(-e_k tau)(1 - f(e_k)) in the form that does not
// overflow for either sign of e_k; with S, also the self-energy of the current iterate at tau_j:
// S_ab(tau_j) = u_a u_b G_ab(tau_j)^2 G_ba(tau_{J-j}).
__global__ void __launch_bounds__(EQ_T) eq_free(const double *e, const double *V, double beta,
                                                int J, int N, double *G0, const double *G,
                                                const double *u, double *S) {
  __shared__ double x[KBE_NMAX], Vs[KBE_NMAX * KBE_NMAX];
  const int j = blockIdx.x, tid = threadIdx.x;
  const double tau = (double)j * beta / J;
  if (tid < N) {
    const double ek = e[tid];
    x[tid] = ek >= 0.0 ? -exp(-ek * tau) / (1.0 + exp(-beta * ek))
                       : -exp(ek * (beta - tau)) / (1.0 + exp(beta * ek));
  }
  if (tid < N * N) Vs[tid] = V[tid];
  __syncthreads();
  if (tid < N * N) {
    const int a = tid / N, b = tid % N;
    double acc = 0.0;
    for (int k = 0; k < N; ++k) acc += Vs[a * N + k] * x[k] * Vs[b * N + k];
    G0[el(j, a, b, N)] = acc;
    if (S) {
      const double g = G[el(j, a, b, N)];
      S[el(j, a, b, N)] = u[a] * u[b] * (g * g) * G[el(J - j, b, a, N)];
    }
  }
}

// The end of a convolution block: tot is the element's sum over l.  COMBINE: Gn = G0 + tot,
// G <- (1 - mix) G + mix Gn in place (no block of the launch reads G), and the block's largest
// |Gn - G| raised into chg (non-negative doubles order like their bit patterns; a NaN wins);
// else out = tot.  red: EQ_T doubles of LDS, free on entry.
template <bool COMBINE>
__device__ __forceinline__ void conv_store(double tot, bool act, size_t i, double *out,
                                           const double *G0, double *G, double mix,
                                           unsigned long long *chg, double *red, int NN) {
  double d = 0.0;
  if (act) {
    if (COMBINE) {
      const double gn = G0[i] + tot, g = G[i];
      d = fabs(gn - g);
      G[i] = (1.0 - mix) * g + mix * gn;
    } else {
      out[i] = tot;
    }
  }
  if (COMBINE) {
    red[threadIdx.x] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = 0.0;
      bool nan = false;
      for (int k = 0; k < NN; ++k) {
        nan |= !(red[k] == red[k]);
        m = red[k] > m ? red[k] : m;
      }
      atomicMax(chg, (unsigned long long)__double_as_longlong(nan ? (double)NAN : m));
    }
  }
}

// out = A * B at tau_j (block j), any N.  Thread (slice s, element (a, b)): the terms
// l = s, s + ns, ... of both parts; the slices are summed in a fixed order.
template <bool COMBINE>
__global__ void __launch_bounds__(EQ_T) eq_conv(const double *A, const double *B,
                                                const double *wf, int J, int N, double *out,
                                                const double *G0, double *G, double mix,
                                                unsigned long long *chg) {
  __shared__ double red[EQ_T];
  const int j = blockIdx.x, tid = threadIdx.x, NN = N * N, ns = EQ_T / NN;
  const int s = tid / NN, e = tid % NN, a = e / N, b = e % N;
  const int64_t ld = (int64_t)J + 1;
  double acc = 0.0;
  if (s < ns) {
    for (int l = s; l <= j; l += ns) {
      const double *Am = A + el(j - l, a, 0, N), *Bl = B + el(l, 0, b, N);
      double v = 0.0;
      for (int c = 0; c < N; ++c) v += Am[c] * Bl[(size_t)c * N];
      acc += wf[j * ld + l] * v;
    }
    for (int l = j + s; l <= J; l += ns) {
      const double *Am = A + el(J + j - l, a, 0, N), *Bl = B + el(l, 0, b, N);
      double v = 0.0;
      for (int c = 0; c < N; ++c) v += Am[c] * Bl[(size_t)c * N];
      acc -= wf[(int64_t)(J - j) * ld + (J - l)] * v;
    }
  }
  red[tid] = acc;
  __syncthreads();
  double tot = 0.0;
  if (tid < NN) {
    tot = red[tid];
    for (int k = 1; k < ns; ++k) tot += red[tid + k * NN];
  }
  __syncthreads();
  conv_store<COMBINE>(tot, tid < NN, el(j, a, b, N), out, G0, G, mix, chg, red, NN);
}

// The same for N = 4 TN: a thread holds a 4 x 4 tile of the output (TN x TN tiles) and walks
// its slice of the ntau + 1 terms (the forward part l = 0..j, then the backward part l = j..J,
// as one sequence); per term the product of the tile's 4 rows of A(tau_m) and 4 columns of
// B(tau_l) in chunks of 4 along the contraction, from 16-byte loads, then one scaled update of
// the tile.  The slices' tiles meet in LDS and are summed in a fixed order.
template <bool COMBINE, int TN>
__global__ void __launch_bounds__(EQ_T) eq_conv4(const double *A, const double *B,
                                                 const double *wf, int J, double *out,
                                                 const double *G0, double *G, double mix,
                                                 unsigned long long *chg) {
  constexpr int N = 4 * TN, NT = TN * TN, NS = EQ_T / NT;
  __shared__ double red[NS * NT * 16];
  const int j = blockIdx.x, tid = threadIdx.x;
  const int s = tid / NT, tt = tid % NT, r0 = 4 * (tt / TN), q0 = 4 * (tt % TN);
  const int64_t ld = (int64_t)J + 1;
  const int nf = j + 1, nterm = J + 2;  // l = 0..j forward, then l = j..J backward
  double acc[4][4] = {};
  if (s < NS) {
    for (int k = s; k < nterm; k += NS) {
      int l, m;
      double w;
      if (k < nf) {
        l = k;
        m = j - l;
        w = wf[j * ld + l];
      } else {
        l = j + (k - nf);
        m = J + j - l;
        w = -wf[(int64_t)(J - j) * ld + (J - l)];
      }
      const double *Am = A + (size_t)m * N * N + (size_t)r0 * N;
      const double *Bl = B + (size_t)l * N * N + q0;
      double t[4][4] = {};
#pragma unroll
      for (int c0 = 0; c0 < N; c0 += 4) {
        double2 x[4][2], y[4][2];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          x[r][0] = *(const double2 *)(Am + r * N + c0);
          x[r][1] = *(const double2 *)(Am + r * N + c0 + 2);
          y[r][0] = *(const double2 *)(Bl + (size_t)(c0 + r) * N);
          y[r][1] = *(const double2 *)(Bl + (size_t)(c0 + r) * N + 2);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double xr[4] = {x[r][0].x, x[r][0].y, x[r][1].x, x[r][1].y};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double yc[4] = {y[c][0].x, y[c][0].y, y[c][1].x, y[c][1].y};
#pragma unroll
            for (int q = 0; q < 4; ++q) t[r][q] += xr[c] * yc[q];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] += w * t[r][q];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[(s * NT + tt) * 16 + r * 4 + q] = acc[r][q];
  }
  __syncthreads();
  const bool act = tid < N * N;
  const int a = act ? tid / N : 0, b = act ? tid % N : 0;
  double tot = 0.0;
  if (act) {
    const int o = ((a >> 2) * TN + (b >> 2)) * 16 + (a & 3) * 4 + (b & 3);
    for (int k = 0; k < NS; ++k) tot += red[k * NT * 16 + o];
  }
  __syncthreads();
  conv_store<COMBINE>(tot, act, el(j, a, b, N), out, G0, G, mix, chg, red, N * N);
}

// A * B for every tau point (COMBINE: the update of G, see conv_store).
template <bool COMBINE>
void launch_conv(const double *A, const double *B, const double *wf, int J, int N, double *out,
                 const double *G0, double *G, double mix, unsigned long long *chg,
                 hipStream_t st) {
  const dim3 g(J + 1), b(EQ_T);
  switch (N) {
    case 4:
      hipLaunchKernelGGL((eq_conv4<COMBINE, 1>), g, b, 0, st, A, B, wf, J, out, G0, G, mix, chg);
      break;
    case 8:
      hipLaunchKernelGGL((eq_conv4<COMBINE, 2>), g, b, 0, st, A, B, wf, J, out, G0, G, mix, chg);
      break;
    case 12:
      hipLaunchKernelGGL((eq_conv4<COMBINE, 3>), g, b, 0, st, A, B, wf, J, out, G0, G, mix, chg);
      break;
    case 16:
      hipLaunchKernelGGL((eq_conv4<COMBINE, 4>), g, b, 0, st, A, B, wf, J, out, G0, G, mix, chg);
      break;
    default:
      hipLaunchKernelGGL(eq_conv<COMBINE>, g, b, 0, st, A, B, wf, J, N, out, G0, G, mix, chg);
  }
}

__global__ void eq_out(const double *G, int64_t tot, kbe_c128 *mat) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < tot) mat[idx] = kbe_c128{G[idx], 0.0};
}

struct EqLayout {
  double *G, *G0, *S, *X, *e, *V;
  unsigned long long *chg;
};

EqLayout eq_layout(void *ws, int N, int ntau) {
  const size_t blk = align256(sizeof(double) * (size_t)ntau * N * N);
  char *p = (char *)ws;
  EqLayout L;
  L.G = (double *)p;
  p += blk;
  L.G0 = (double *)p;
  p += blk;
  L.S = (double *)p;
  p += blk;
  L.X = (double *)p;
  p += blk;
  L.e = (double *)p;
  p += align256(sizeof(double) * N);
  L.V = (double *)p;
  p += align256(sizeof(double) * N * N);
  L.chg = (unsigned long long *)p;
  return L;
}

}  // namespace

size_t equilibrium_ws_bytes(int N, int ntau) {
  return 4 * align256(sizeof(double) * (size_t)ntau * N * N) + align256(sizeof(double) * N) +
         align256(sizeof(double) * N * N) + 256;
}

hipError_t launch_equilibrium(int N, int ntau, double beta, const double *wf, const double *h0,
                              const double *u, double mu, double mix, double tol, int maxit,
                              kbe_c128 *mat, void *ws, hipStream_t st, int *iterations,
                              double *change) {
  const EqLayout L = eq_layout(ws, N, ntau);
  const int J = ntau - 1;
  const int64_t tot = (int64_t)ntau * N * N;
  const unsigned eb = (unsigned)((tot + 255) / 256);
  // the starting point: the free function of h0 - mu
  hipLaunchKernelGGL(eq_eig, dim3(1), dim3(EQ_T), 0, st, h0, u, mu, L.G, J, N, 0, 0, L.e, L.V,
                     L.chg);
  hipLaunchKernelGGL(eq_free, dim3(ntau), dim3(EQ_T), 0, st, L.e, L.V, beta, J, N, L.G,
                     nullptr, nullptr, nullptr);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  double d = INFINITY;
  int it = 0;
  while (it < maxit) {
    ++it;
    hipLaunchKernelGGL(eq_eig, dim3(1), dim3(EQ_T), 0, st, h0, u, mu, L.G, J, N, 1, 1, L.e,
                       L.V, L.chg);
    hipLaunchKernelGGL(eq_free, dim3(ntau), dim3(EQ_T), 0, st, L.e, L.V, beta, J, N, L.G0,
                       L.G, u, L.S);
    launch_conv<false>(L.S, L.G, wf, J, N, L.X, nullptr, nullptr, 0.0, nullptr, st);
    launch_conv<true>(L.G0, L.X, wf, J, N, nullptr, L.G0, L.G, mix, L.chg, st);
    unsigned long long bits = 0;
    err = hipMemcpyAsync(&bits, L.chg, sizeof bits, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) return err;
    memcpy(&d, &bits, sizeof d);
    if (!std::isfinite(d) || d < tol) break;
  }
  hipLaunchKernelGGL(eq_out, dim3(eb), dim3(256), 0, st, L.G, tot, mat);
  *iterations = it;
  *change = d;
  return hipGetLastError();
}

}  // namespace kbe
