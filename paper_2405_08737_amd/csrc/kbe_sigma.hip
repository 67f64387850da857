// Second-Born self-energy row (Eq. SE of arXiv:2405.08737, local interaction) and its adjoint.
//
// For U_{ijkl} = u_i d_ij d_jk d_kl, Eq. SE reduces elementwise to
//   Sigma^<_ij(t,t') = u_i u_j G^<_ij(t,t')^2 G^>_ji(t',t)
//   Sigma^>_ij(t,t') = u_i u_j G^>_ij(t,t')^2 G^<_ji(t',t)
//   Sigma^]_ij(t,tau) = u_i u_j G^]_ij(t,tau)^2 conj(G^]_ij(t,beta-tau))
// One thread per element of the row (s, i, j) or (tau_l, i, j).  With a = kp[s][n]_ji
// (= G^<(t_s,t_n)_ji) and, for s < n, R = kp[n][s]_ij (= G^R(t_n,t_s)_ij):
//   G^<(t_n,t_s)_ij = -conj(a),  G^>(t_n,t_s)_ij = g = R - conj(a),  G^>(t_s,t_n)_ji = -conj(g).
// At s = n the stored diagonal block D = kp[n][n] and r = rdiag[n] are read directly:
//   G^<_ij = D_ij, G^>_ij = r_ij + D_ij, G^<_ji = D_ji, G^>_ji = r_ji + D_ji.
#include "kbe_dev.h"
#include "kbe_internal.h"

namespace kbe {

struct SigArgs {
  int N, ntau, J, n;
  int64_t ldt;
  const kbe_c128 *kp, *rdiag, *tv;
  const double *u;
};

// Element idx of the row at t_n: the first (n+1) N^2 are Sigma^R and Sigma^< at (t_n, t_s), the
// next ntau N^2 are Sigma^](t_n, tau_l).
__device__ __forceinline__ void sigma_row_elem(const SigArgs &a, int64_t idx, kbe_c128 *ret,
                                               kbe_c128 *les, kbe_c128 *stv) {
  const int64_t E = (int64_t)a.N * a.N;
  const int64_t nrt = (int64_t)(a.n + 1) * E;
  if (idx < nrt) {
    const int s = (int)(idx / E), e = (int)(idx % E), i = e / a.N, j = e % a.N;
    const double U = a.u[i] * a.u[j];
    const cd z1 = ld(a.kp + ((int64_t)s * a.ldt + a.n) * E + j * a.N + i);  // G^<(s,n)_ji
    cd sl, sg;
    if (s < a.n) {
      const cd R = ld(a.kp + ((int64_t)a.n * a.ldt + s) * E + e);
      const cd L = -cj(z1);
      const cd g = R + L;
      sl = U * (L * L * (-cj(g)));
      sg = U * (g * g * z1);
    } else {
      const kbe_c128 *D = a.kp + ((int64_t)a.n * a.ldt + a.n) * E;
      const kbe_c128 *r = a.rdiag + (int64_t)a.n * E;
      const cd Dij = ld(D + e), rij = ld(r + e), rji = ld(r + j * a.N + i);
      const cd gij = rij + Dij, gji = rji + z1;
      sl = U * (Dij * Dij * gji);
      sg = U * (gij * gij * z1);
    }
    st(les + s * E + e, sl);
    st(ret + s * E + e, sg - sl);
  } else if (idx < nrt + (int64_t)a.ntau * E) {
    const int64_t k = idx - nrt;
    const int l = (int)(k / E), e = (int)(k % E), i = e / a.N, j = e % a.N;
    const double U = a.u[i] * a.u[j];
    const cd x = ld(a.tv + ((int64_t)a.n * a.ntau + l) * E + e);
    const cd y = ld(a.tv + ((int64_t)a.n * a.ntau + (a.J - l)) * E + e);
    st(stv + (int64_t)l * E + e, U * (x * x * cj(y)));
  }
}

__global__ void __launch_bounds__(256) sigma_row_kernel(SigArgs a, kbe_c128 *ret, kbe_c128 *les,
                                                        kbe_c128 *stv) {
  sigma_row_elem(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, ret, les, stv);
}

// Rows of many systems: blockIdx.y is the item; the item's workgroups stride over its elements.
__global__ void __launch_bounds__(256) sigma_batch_kernel(const kbe_sigma_batch_item *items) {
  const kbe_sigma_batch_item it = items[blockIdx.y];
  const SigArgs a{it.N, it.ntau, it.ntau - 1, it.n, it.ldt, it.kp, it.rdiag, it.tv, it.u};
  const int64_t tot = (int64_t)(it.n + 1 + it.ntau) * it.N * it.N;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += stride)
    sigma_row_elem(a, idx, it.ret, it.les, it.stv);
}

hipError_t launch_sigma_batch(const kbe_sigma_batch_item *items_dev, int count, int64_t max_elems,
                              hipStream_t st) {
  // workgroups per item: enough for the longest row at four elements per thread, at most 256
  int64_t per = (max_elems + 4 * 256 - 1) / (4 * 256);
  per = per < 1 ? 1 : (per > 256 ? 256 : per);
  constexpr int YMAX = 32768;  // items per launch (grid y)
  for (int off = 0; off < count; off += YMAX) {
    const int c = count - off < YMAX ? count - off : YMAX;
    hipLaunchKernelGGL(sigma_batch_kernel, dim3((unsigned)per, (unsigned)c), dim3(256), 0, st,
                       items_dev + off);
  }
  return hipGetLastError();
}

// out = a + b elementwise (out may be a or b).
__global__ void __launch_bounds__(256) add_blocks_kernel(const kbe_c128 *a, const kbe_c128 *b,
                                                         kbe_c128 *out, int64_t cnt) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < cnt) st(out + idx, ld(a + idx) + ld(b + idx));
}

hipError_t launch_add_blocks(const kbe_c128 *a, const kbe_c128 *b, kbe_c128 *out, int64_t cnt,
                             hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_blocks_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, a,
                     b, out, cnt);
  return hipGetLastError();
}

hipError_t launch_sigma_row(const kbe_green *G, const double *u, int n, const kbe_sigma_row *out,
                            hipStream_t st) {
  SigArgs a{G->N, G->ntau, G->ntau - 1, n, G->ldt, G->kp, G->rdiag, G->tv, u};
  const int64_t tot = (int64_t)(n + 1 + G->ntau) * G->N * G->N;
  hipLaunchKernelGGL(sigma_row_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a,
                     out->ret, out->les, out->tv);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Full mode: Sigma for every time pair, in KP storage like G (Sigma^< on and above the diagonal,
// Sigma^R = Sigma^> - Sigma^< below it, the one-sided Sigma^R(t,t) in rdiag, Sigma^] in tv).  One
// thread per stored element; every value comes from the formula at its own arguments, with G
// read through the storage symmetries:
//   G^<(a,b) = kp[a][b] (a <= b), -kp[b][a]^dagger (a > b)
//   G^>(a,b) = G^R(a,b) + G^<(a,b) (a >= b; G^R from kp[a][b], or rdiag[a] at a = b),
//              -G^>(b,a)^dagger (a < b).
// ---------------------------------------------------------------------------------------------
struct FullArgs {
  SigArgs a;
  int nt;
  int64_t sldt;
  kbe_c128 *skp, *srd, *stv;
};

__device__ __forceinline__ cd g_les(const SigArgs &a, int x, int y, int i, int j) {
  const int64_t E = (int64_t)a.N * a.N;
  return x <= y ? ld(a.kp + ((int64_t)x * a.ldt + y) * E + i * a.N + j)
                : -cj(ld(a.kp + ((int64_t)y * a.ldt + x) * E + j * a.N + i));
}
__device__ __forceinline__ cd g_gtr(const SigArgs &a, int x, int y, int i, int j) {
  const int64_t E = (int64_t)a.N * a.N;
  if (x < y) {
    const cd r = ld(a.kp + ((int64_t)y * a.ldt + x) * E + j * a.N + i);  // G^R(y,x)_ji
    return -cj(r + g_les(a, y, x, j, i));
  }
  const cd r = x == y ? ld(a.rdiag + (int64_t)x * E + i * a.N + j)
                      : ld(a.kp + ((int64_t)x * a.ldt + y) * E + i * a.N + j);
  return r + g_les(a, x, y, i, j);
}

__global__ void __launch_bounds__(256) sigma_full_kernel(FullArgs f) {
  const SigArgs &a = f.a;
  const int N = a.N;
  const int64_t E = (int64_t)N * N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nkp = (int64_t)f.nt * f.nt * E, nrd = (int64_t)f.nt * E;
  if (idx < nkp + nrd) {
    const bool diag = idx >= nkp;
    const int64_t k = diag ? idx - nkp : idx;
    const int x = diag ? (int)(k / E) : (int)(k / E / f.nt);
    const int y = diag ? x : (int)(k / E % f.nt);
    const int e = (int)(k % E), i = e / N, j = e % N;
    const double U = a.u[i] * a.u[j];
    const cd lxy = g_les(a, x, y, i, j), gxy = g_gtr(a, x, y, i, j);
    const cd lyx = g_les(a, y, x, j, i), gyx = g_gtr(a, y, x, j, i);
    const cd sl = U * (lxy * lxy * gyx), sg = U * (gxy * gxy * lyx);
    if (diag) st(f.srd + (int64_t)x * E + e, sg - sl);
    else st(f.skp + ((int64_t)x * f.sldt + y) * E + e, x <= y ? sl : sg - sl);
  } else if (idx < nkp + nrd + (int64_t)f.nt * a.ntau * E) {
    const int64_t k = idx - nkp - nrd;
    const int x = (int)(k / E / a.ntau), l = (int)(k / E % a.ntau), e = (int)(k % E);
    const int i = e / N, j = e % N;
    const double U = a.u[i] * a.u[j];
    const cd v = ld(a.tv + ((int64_t)x * a.ntau + l) * E + e);
    const cd w = ld(a.tv + ((int64_t)x * a.ntau + (a.J - l)) * E + e);
    st(f.stv + ((int64_t)x * a.ntau + l) * E + e, U * (v * v * cj(w)));
  }
}

hipError_t launch_sigma_full(const kbe_green *G, const double *u, const kbe_green *S,
                             hipStream_t st) {
  FullArgs f{{G->N, G->ntau, G->ntau - 1, 0, G->ldt, G->kp, G->rdiag, G->tv, u}, G->nt, S->ldt,
             S->kp, S->rdiag, S->tv};
  const int64_t E = (int64_t)G->N * G->N;
  const int64_t tot = ((int64_t)G->nt * G->nt + G->nt + (int64_t)G->nt * G->ntau) * E;
  hipLaunchKernelGGL(sigma_full_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, f);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Adjoint.  Complex gradients follow PyTorch's convention (dL/dRe + i dL/dIm); for W(z, conj z)
// the gradient is  conj(gW) dW/dconj(z) + gW conj(dW/dz).  With G1 = gret and G2 = gles - gret
// (Sigma^> enters ret with +, Sigma^< enters les with + and ret with -), for s < n:
//   Sigma^< = U conj(z1)^2 (z1 - conj(z2)),  Sigma^> = U g^2 z1,  g = z2 - conj(z1)
//   d/dz1 :  2U conj(G2) conj(z1)(z1 - conj(z2)) + U G2 z1^2 - 2U conj(G1) g z1 + U G1 conj(g)^2
//   d/dz2 : -U conj(G2) conj(z1)^2 + 2U G1 conj(g) conj(z1)
// Every storage entry is owned by exactly one thread (the diagonal block and the tau row are
// gathered from the two elements that read an entry), so gradients are added without races.
// The interaction gradient gu_k = sum Re(conj(gW) dW/du_k) is reduced deterministically in two
// stages through the workspace.
// ---------------------------------------------------------------------------------------------
struct SigVjpArgs {
  SigArgs a;
  const kbe_c128 *gret, *gles, *gstv;
  kbe_c128 *gkp, *grdiag, *gtv;
  double *part;  // [blocks][N]
};

__global__ void __launch_bounds__(256) sigma_row_vjp_kernel(SigVjpArgs v) {
  const SigArgs &a = v.a;
  const int N = a.N;
  const int64_t E = (int64_t)N * N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nrt = (int64_t)(a.n + 1) * E;
  double contrib = 0.0;
  int ci = 0, cjx = 0;
  if (idx < nrt) {
    const int s = (int)(idx / E), e = (int)(idx % E), i = e / N, j = e % N;
    const double U = a.u[i] * a.u[j];
    ci = i;
    cjx = j;
    const cd G1 = ld(v.gret + s * E + e);
    const cd G2 = ld(v.gles + s * E + e) - G1;
    if (s < a.n) {
      kbe_c128 *pz1 = v.gkp + ((int64_t)s * a.ldt + a.n) * E + j * N + i;
      kbe_c128 *pz2 = v.gkp + ((int64_t)a.n * a.ldt + s) * E + e;
      const cd z1 = ld(a.kp + ((int64_t)s * a.ldt + a.n) * E + j * N + i);
      const cd z2 = ld(a.kp + ((int64_t)a.n * a.ldt + s) * E + e);
      const cd g = z2 - cj(z1);
      const cd w = z1 - cj(z2);
      const cd c1 = cj(z1);
      const cd gz1 = (2.0 * U) * (cj(G2) * c1 * w) + U * (G2 * z1 * z1) -
                     (2.0 * U) * (cj(G1) * g * z1) + U * (G1 * cj(g) * cj(g));
      const cd gz2 = (2.0 * U) * (G1 * cj(g) * c1) - U * (cj(G2) * c1 * c1);
      st(pz1, ld(pz1) + gz1);
      st(pz2, ld(pz2) + gz2);
      const cd Xl = c1 * c1 * w, Xg = g * g * z1;
      contrib = (cj(G2) * Xl).re + (cj(G1) * Xg).re;
    } else {
      const kbe_c128 *D = a.kp + ((int64_t)a.n * a.ldt + a.n) * E;
      const kbe_c128 *r = a.rdiag + (int64_t)a.n * E;
      const int et = j * N + i;
      const cd Dij = ld(D + e), Dji = ld(D + et), rij = ld(r + e), rji = ld(r + et);
      // element (i,j): reads D_ij, D_ji, r_ij, r_ji
      const cd toD = G2 * cj(2.0 * U * (Dij * (rji + Dji))) + G1 * cj(2.0 * U * ((rij + Dij) * Dji));
      const cd toR = G1 * cj(2.0 * U * ((rij + Dij) * Dji));
      // element (j,i): its "ji" entries are D_ij, r_ij
      const cd H1 = ld(v.gret + s * E + et);
      const cd H2 = ld(v.gles + s * E + et) - H1;
      const cd fromD = H2 * cj(U * (Dji * Dji)) + H1 * cj(U * ((rji + Dji) * (rji + Dji)));
      const cd fromR = H2 * cj(U * (Dji * Dji));
      kbe_c128 *pD = v.gkp + ((int64_t)a.n * a.ldt + a.n) * E + e;
      kbe_c128 *pr = v.grdiag + (int64_t)a.n * E + e;
      st(pD, ld(pD) + toD + fromD);
      st(pr, ld(pr) + toR + fromR);
      contrib = (cj(G2) * (Dij * Dij * (rji + Dji))).re + (cj(G1) * ((rij + Dij) * (rij + Dij) * Dji)).re;
    }
  } else if (idx < nrt + (int64_t)a.ntau * E) {
    const int64_t k = idx - nrt;
    const int l = (int)(k / E), e = (int)(k % E), i = e / N, j = e % N;
    const double U = a.u[i] * a.u[j];
    ci = i;
    cjx = j;
    const cd x = ld(a.tv + ((int64_t)a.n * a.ntau + l) * E + e);
    const cd y = ld(a.tv + ((int64_t)a.n * a.ntau + (a.J - l)) * E + e);
    const cd gl = ld(v.gstv + (int64_t)l * E + e);
    const cd gm = ld(v.gstv + (int64_t)(a.J - l) * E + e);
    kbe_c128 *px = v.gtv + ((int64_t)a.n * a.ntau + l) * E + e;
    st(px, ld(px) + gl * cj(2.0 * U * (x * cj(y))) + cj(gm) * (U * (y * y)));
    contrib = (cj(gl) * (x * x * cj(y))).re;
  }
  // stage 1 of the interaction gradient: per-block partial sums in a fixed order.  Each entry
  // adds u_j c to gu_i and u_i c to gu_j; for every orbital q the wave sums its lanes' shares by
  // a fixed butterfly, then the four waves' sums are added in order.
  __shared__ double ws[4][KBE_NMAX];
  const double sa = a.u[cjx] * contrib, sb = a.u[ci] * contrib;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q = 0; q < N; ++q) {
    double x = (ci == q ? sa : 0.0) + (cjx == q ? sb : 0.0);
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) ws[wv][q] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < N) {
    const int q = threadIdx.x;
    v.part[(int64_t)blockIdx.x * N + q] = ((ws[0][q] + ws[1][q]) + ws[2][q]) + ws[3][q];
  }
}

// Stage 2: gu[q] += sum over blocks of part[b][q].  256 threads: thread (q, r) sums the blocks
// b = r, r+16, ... in order, then the 16 partial sums of each q are added in a fixed tree.
__global__ void __launch_bounds__(256) gu_reduce_kernel(const double *part, int nblk, int N,
                                                        double *gu) {
  __shared__ double red[16][17];
  const int q = threadIdx.x & 15, r = threadIdx.x >> 4;
  double acc = 0.0;
  if (q < N)
    for (int b = r; b < nblk; b += 16) acc += part[(int64_t)b * N + q];
  red[r][q] = acc;
  __syncthreads();
  for (int h = 8; h > 0; h >>= 1) {
    if (r < h) red[r][q] += red[r + h][q];
    __syncthreads();
  }
  if (r == 0 && q < N) gu[q] += red[0][q];
}

static int64_t sigma_vjp_blocks(int N, int n, int ntau) {
  return ((int64_t)(n + 1 + ntau) * N * N + 255) / 256;
}

size_t sigma_vjp_ws_bytes(int N, int n, int ntau) {
  return sizeof(double) * (size_t)sigma_vjp_blocks(N, n, ntau) * N;
}

hipError_t launch_sigma_row_vjp(const kbe_green *G, const double *u, int n,
                                const kbe_sigma_row *gS, const kbe_green *gG, double *gu,
                                void *ws, hipStream_t st) {
  SigVjpArgs v;
  v.a = SigArgs{G->N, G->ntau, G->ntau - 1, n, G->ldt, G->kp, G->rdiag, G->tv, u};
  v.gret = gS->ret;
  v.gles = gS->les;
  v.gstv = gS->tv;
  v.gkp = gG->kp;
  v.grdiag = gG->rdiag;
  v.gtv = gG->tv;
  v.part = (double *)ws;
  const int64_t nblk = sigma_vjp_blocks(G->N, n, G->ntau);
  hipLaunchKernelGGL(sigma_row_vjp_kernel, dim3((unsigned)nblk), dim3(256), 0, st, v);
  hipLaunchKernelGGL(gu_reduce_kernel, dim3(1), dim3(256), 0, st, (const double *)ws, (int)nblk,
                     G->N, gu);
  return hipGetLastError();
}

}  // namespace kbe
