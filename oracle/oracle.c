/*
 * CPU ORACLE for the Kadanoff-Baym history-integral path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, loads or calls
 * this file; only the test-suite, the package's smoke check and the benchmark's
 * CPU-baseline leg use it.  It is plain, slow, FP64 C written to be checked
 * against the paper by eye: loops in the paper's order, no blocking, no fusion,
 * no reordering.  Complex arithmetic uses C99 double complex.
 *
 * Paper: T. Blommel, D. J. Gardner, C. S. Woodward, E. Gull, "Adaptive Time
 * Stepping for the Two-Time Integro-Differential Kadanoff-Baym Equations",
 * arXiv:2405.08737.
 *
 * Storage (this file's own statement; the GPU side documents its own):
 *   kp    [nt][ldt][N][N]: kp[a][b] = G^<(t_a,t_b) for a <= b, G^R(t_a,t_b) for a > b
 *   rdiag [nt][N][N]     : G^R(t_a,t_a)
 *   tv    [nt][ntau][N][N]: G^](t_m,tau_j)          (mixed component)
 *   mat   [ntau][N][N]   : G^M(tau_j), j=0 holds G^M(0+), j=ntau-1 holds G^M(beta-)
 *   Self-energy rows at t_n: ret[s] = Sigma^R(t_n,t_s), les[s] = Sigma^<(t_n,t_s)
 *   (s = 0..n), stv[j] = Sigma^](t_n,tau_j).
 *
 * Every function states the passage of the paper it follows.  Readings of
 * places where the paper is silent are marked READING.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define BLK(p, idx, N) ((p) + (int64_t)(idx) * (N) * (N))

/* ------------------------------------------------------------------------- */
/* Quadrature weights (Sec. "Adaptive History Integration", Eq. weights and   */
/* the weight-row recursion that follows it).                                */
/* ------------------------------------------------------------------------- */

/* Gauss-Legendre rule with m points on [-1,1]: nodes are the roots of the
 * Legendre polynomial P_m, found by Newton's method on the three-term
 * recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}; weights
 * 2 / ((1-x^2) P_m'(x)^2).  (Textbook rule; used here only as an exact
 * integrator for polynomials of degree <= 2m-1.) */
void orc_gauss_legendre(int m, double *x, double *w) {
  for (int i = 0; i < m; ++i) {
    double z = cos(M_PI * (i + 0.75) / (m + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < m; ++k) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      /* p1 = P_m(z), p0 = P_{m-1}(z) */
      dp = m * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < m; ++k) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = m * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* Local weights of interval p (the integral over [t_{p-1}, t_p]) using the k
 * most recent nodes x_j = t[p-k+1+j], j = 0..k-1 (Eq. weights).  By
 * definition lam_j is the integral of the Lagrange basis polynomial l_j of
 * those nodes over the interval, because integrating the interpolant
 * sum_j g_j l_j(t) is what Eq. weights does.  This oracle evaluates that
 * definition directly: l_j is formed as its product formula in the scaled
 * variable y = (t - t_p)/h_p and integrated with a Gauss-Legendre rule that
 * is exact for its degree k-1.  (The paper instead solves a Vandermonde
 * system; both give the same numbers, and a test checks that.) */
void orc_local_weights(const double *t, int p, int k, double *lam) {
  double h = t[p] - t[p - 1];
  double y[64];
  for (int j = 0; j < k; ++j) y[j] = (t[p - k + 1 + j] - t[p]) / h;
  int m = (k + 1) / 2 + 1;
  double gx[64], gw[64];
  orc_gauss_legendre(m, gx, gw);
  for (int j = 0; j < k; ++j) {
    double acc = 0.0;
    for (int g = 0; g < m; ++g) {
      double yy = 0.5 * (gx[g] - 1.0); /* [-1,1] -> [-1,0] */
      double l = 1.0;
      for (int i = 0; i < k; ++i)
        if (i != j) l *= (yy - y[i]) / (y[j] - y[i]);
      acc += 0.5 * gw[g] * l;
    }
    lam[j] = h * acc;
  }
}

/* Composite weight matrix w[n][s] (row-major, nt x nt) such that
 * sum_s w[n][s] g(t_s) approximates the integral of g over [0, t_n].
 * Row recursion of the paper: row n = row n-1 plus the local weights of
 * interval n placed on its nodes.  READING: interval p uses
 * k_p = min(order[p], p+1) nodes (all available points during start-up);
 * row 0 is zero. */
void orc_weights(const double *t, const int32_t *order, int nt, double *w) {
  memset(w, 0, sizeof(double) * (size_t)nt * nt);
  double lam[64];
  for (int n = 1; n < nt; ++n) {
    for (int s = 0; s < nt; ++s) w[(int64_t)n * nt + s] = w[(int64_t)(n - 1) * nt + s];
    int k = order[n] < n + 1 ? order[n] : n + 1;
    orc_local_weights(t, n, k, lam);
    for (int j = 0; j < k; ++j) w[(int64_t)n * nt + (n - k + 1 + j)] += lam[j];
  }
}

/* Weights of the integral over [x_lo, x_hi] on the nodes x_lo..x_hi of a grid
 * that is known in full (the imaginary-time grid).  Every interval p in
 * (lo, hi] is integrated with the Lagrange rule of Eq. weights on
 * kk = min(k, hi-lo+1) nodes; the window ends at the interval's right node
 * p, shifted right where it would leave the piece: first node
 * a = clamp(p-kk+1, lo, hi-kk+1).  Output wrow[lo..hi]; other entries 0. */
static void piece_weights(const double *x, int nx, int lo, int hi, int k, double *wrow) {
  for (int l = 0; l < nx; ++l) wrow[l] = 0.0;
  int kk = k < hi - lo + 1 ? k : hi - lo + 1;
  double lam[64], xs[64];
  for (int p = lo + 1; p <= hi; ++p) {
    int a = p - kk + 1;
    if (a < lo) a = lo;
    if (a > hi - kk + 1) a = hi - kk + 1;
    /* orc_local_weights integrates over [x_{q-1}, x_q] with nodes ending at q;
     * here the interval is [x_{p-1}, x_p] and the nodes are x_a..x_{a+kk-1}. */
    double h = x[p] - x[p - 1];
    int m = (kk + 1) / 2 + 1;
    double gx[64], gw[64];
    orc_gauss_legendre(m, gx, gw);
    for (int j = 0; j < kk; ++j) xs[j] = (x[a + j] - x[p]) / h;
    for (int j = 0; j < kk; ++j) {
      double acc = 0.0;
      for (int g = 0; g < m; ++g) {
        double yy = 0.5 * (gx[g] - 1.0);
        double l = 1.0;
        for (int i = 0; i < kk; ++i)
          if (i != j) l *= (yy - xs[i]) / (xs[j] - xs[i]);
        acc += 0.5 * gw[g] * l;
      }
      lam[j] = h * acc;
    }
    for (int j = 0; j < kk; ++j) wrow[a + j] += lam[j];
  }
}

/* Imaginary-time weights.  READING (the paper takes its tau points and
 * convolution tensors from the DLR package, which is not used here): tau is
 * the uniform grid tau_j = j beta / J, J = ntau-1, and each tau integral uses
 * the Lagrange rule of Eq. weights with tau_order nodes per interval, on
 * windows kept inside the range of integration (piece_weights).
 *   wf[j][l]: weights of the integral over [0, tau_j]   (nodes l <= j)
 *   wb[j][l]: weights of the integral over [tau_j, beta] (nodes l >= j),
 *             obtained by applying the same construction to the reversed
 *             grid u = beta - tau and mapping the nodes back
 *   wfull[l]: weights of the integral over [0, beta], the average of the
 *             forward and backward full-range rules, so that it is symmetric
 *             under l -> J-l. */
void orc_tau_weights(double beta, int ntau, int tau_order, double *wf, double *wb, double *wfull) {
  int J = ntau - 1;
  double *tau = malloc(sizeof(double) * ntau);
  double *u = malloc(sizeof(double) * ntau);
  double *row = malloc(sizeof(double) * ntau);
  for (int j = 0; j < ntau; ++j) tau[j] = beta * j / J;
  /* reversed grid: u_q = beta - tau_{J-q}, q = 0..J (increasing from 0); node u_q is tau_{J-q} */
  for (int q = 0; q < ntau; ++q) u[q] = beta - tau[J - q];
  u[0] = 0.0;
  for (int j = 0; j < ntau; ++j) {
    piece_weights(tau, ntau, 0, j, tau_order, wf + (int64_t)j * ntau);
    /* [tau_j, beta] is u in [0, beta - tau_j] = [u_0, u_{J-j}] */
    piece_weights(u, ntau, 0, J - j, tau_order, row);
    for (int l = 0; l < ntau; ++l) wb[(int64_t)j * ntau + l] = row[J - l];
  }
  for (int l = 0; l < ntau; ++l)
    wfull[l] = 0.5 * (wf[(int64_t)J * ntau + l] + wb[(int64_t)0 * ntau + l]);
  free(tau);
  free(u);
  free(row);
}

/* ------------------------------------------------------------------------- */
/* Keldysh components from the storage (Sec. "Kadanoff Baym Equations":       */
/* lesser/greater symmetry, G^> - G^< = G^R for t > t'; Sec. "Implementation" */
/* for storing one side of the diagonal).                                    */
/* ------------------------------------------------------------------------- */

typedef struct {
  int N, nt, ntau;
  int64_t ldt;
  const cplx *kp, *rdiag, *tv, *mat;
} green;

static const cplx *kp_blk(const green *g, int a, int b) {
  return g->kp + ((int64_t)a * g->ldt + b) * g->N * g->N;
}

/* G^<(t_a,t_b): stored for a <= b; for a > b use G^<(t,t') = -G^<(t',t)^dagger. */
static void get_les(const green *g, int a, int b, cplx *out) {
  int N = g->N;
  if (a <= b) {
    memcpy(out, kp_blk(g, a, b), sizeof(cplx) * N * N);
  } else {
    const cplx *x = kp_blk(g, b, a);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) out[i * N + j] = -conj(x[j * N + i]);
  }
}

/* G^R(t_a,t_b) for a >= b: stored below the diagonal, equal-time value in rdiag. */
static void get_ret(const green *g, int a, int b, cplx *out) {
  int N = g->N;
  const cplx *x = (a == b) ? BLK(g->rdiag, a, N) : kp_blk(g, a, b);
  memcpy(out, x, sizeof(cplx) * N * N);
}

/* G^>(t_a,t_b): for a >= b, G^> = G^R + G^< (definition of G^R); for a < b
 * use G^>(t,t') = -G^>(t',t)^dagger. */
static void get_gtr(const green *g, int a, int b, cplx *out) {
  int N = g->N;
  if (a >= b) {
    cplx r[256], l[256];
    get_ret(g, a, b, r);
    get_les(g, a, b, l);
    for (int e = 0; e < N * N; ++e) out[e] = r[e] + l[e];
  } else {
    cplx x[256];
    get_gtr(g, b, a, x);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) out[i * N + j] = -conj(x[j * N + i]);
  }
}

/* ------------------------------------------------------------------------- */
/* Second-Born (GF2) self-energy, Eq. SE, for a local interaction            */
/* U_{ijkl} = u_i delta_ij delta_jk delta_kl.  Then U^Ex_{jabc} = u_j for    */
/* a=b=c=j and Eq. SE reduces to                                             */
/*   Sigma^<>_ij(t,t') = u_i u_j G^<>_ij(t,t')^2 G^><_ji(t',t)               */
/*   Sigma^]_ij(t,tau) = u_i u_j G^]_ij(t,tau)^2 G^[_ji(tau,t),              */
/* with G^[(tau,t) = G^](t,beta-tau)^dagger.  (A test checks the reduction   */
/* against the general four-index formula by brute force.)                   */
/* ------------------------------------------------------------------------- */

/* Sigma^< and Sigma^> at an arbitrary pair (t_a, t_b). */
void orc_sigma_pair(int N, int nt, int ntau, int64_t ldt, const cplx *kp, const cplx *rdiag,
                    const double *u, int a, int b, cplx *les, cplx *gtr) {
  green g = {N, nt, ntau, ldt, kp, rdiag, NULL, NULL};
  cplx lab[256], lba[256], gab[256], gba[256];
  get_les(&g, a, b, lab);
  get_les(&g, b, a, lba);
  get_gtr(&g, a, b, gab);
  get_gtr(&g, b, a, gba);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      les[i * N + j] = u[i] * u[j] * lab[i * N + j] * lab[i * N + j] * gba[j * N + i];
      gtr[i * N + j] = u[i] * u[j] * gab[i * N + j] * gab[i * N + j] * lba[j * N + i];
    }
}

/* Self-energy row at t_n: ret[s] = Sigma^R(t_n,t_s) = Sigma^> - Sigma^< for
 * s <= n (READING: at s = n the one-sided value Sigma^>(t,t) - Sigma^<(t,t)),
 * les[s] = Sigma^<(t_n,t_s), stv[l] = Sigma^](t_n,tau_l).  The tau grid is
 * symmetric, so beta - tau_l = tau_{J-l}. */
void orc_sigma_row(int N, int nt, int ntau, int64_t ldt, const cplx *kp, const cplx *rdiag,
                   const cplx *tv, const double *u, int n, cplx *ret, cplx *les, cplx *stv) {
  for (int s = 0; s <= n; ++s) {
    cplx l[256], gg[256];
    orc_sigma_pair(N, nt, ntau, ldt, kp, rdiag, u, n, s, l, gg);
    for (int e = 0; e < N * N; ++e) {
      les[(int64_t)s * N * N + e] = l[e];
      ret[(int64_t)s * N * N + e] = gg[e] - l[e];
    }
  }
  int J = ntau - 1;
  for (int l = 0; l < ntau; ++l) {
    const cplx *x = tv + ((int64_t)n * ntau + l) * N * N;
    const cplx *y = tv + ((int64_t)n * ntau + (J - l)) * N * N;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        cplx gmix = x[i * N + j];
        cplx gbar = conj(y[i * N + j]); /* G^[_ji(tau_l, t_n) = conj(G^]_ij(t_n, beta - tau_l)) */
        stv[((int64_t)l * N + i) * N + j] = u[i] * u[j] * gmix * gmix * gbar;
      }
  }
}

/* ------------------------------------------------------------------------- */
/* History integrals (Eq. KBE2, lesser form, at t = t_n, t' = t_m; and the    */
/* history terms of Eq. KBE3 at t = t_n).                                    */
/* ------------------------------------------------------------------------- */

/* out += c * A * op(B), op = identity (hb = 0) or conjugate transpose (hb = 1). */
static void mm_acc(int N, cplx *out, cplx c, const cplx *A, const cplx *B, int hb) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      cplx acc = 0;
      for (int k = 0; k < N; ++k) {
        cplx b = hb ? conj(B[j * N + k]) : B[k * N + j];
        acc += A[i * N + k] * b;
      }
      out[i * N + j] += c * acc;
    }
}

/* out += c * A^dagger * B. */
static void mm_acc_hn(int N, cplx *out, cplx c, const cplx *A, const cplx *B) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      cplx acc = 0;
      for (int k = 0; k < N; ++k) acc += conj(A[k * N + i]) * B[k * N + j];
      out[i * N + j] += c * acc;
    }
}

/* F_GREATER: the greater form of Eq. KBE2, G^>(t_s,t_m) in I^R and Sigma^> = Sigma^R + Sigma^<
 * (the same self-energy row) in I^<; I^] and J^] do not depend on the form. */
enum { F_IR = 1, F_IL = 2, F_ITV = 4, F_JTV = 8, F_GREATER = 1024 };

/* Index of the tau point beta - tau_j (the grid is symmetric). */
static int tau_mirror(int ntau, int j) { return ntau - 1 - j; }

/* Forward history integrals at row n for outputs m in [m0, m1):
 *   IR(m)  = int_0^{t_n} Sigma^R(t_n,s) G^<(s,t_m) ds
 *          ~ sum_{s=0}^{n} w[n][s] Sigma^R(t_n,t_s) G^<(t_s,t_m)
 *   IL(m)  = int_0^{t_m} Sigma^<(t_n,s) G^A(s,t_m) ds,  G^A(s,t') = G^R(t',s)^dagger
 *          ~ sum_{s=0}^{m} w[m][s] Sigma^<(t_n,t_s) G^R(t_m,t_s)^dagger
 *          (READING: the equal-time endpoint takes the one-sided G^R(t,t))
 *   Itv(m) = -i int_0^beta Sigma^](t_n,tau) G^[(tau,t_m) dtau
 *          ~ -i sum_j wfull[j] Sigma^](t_n,tau_j) G^](t_m,beta-tau_j)^dagger
 *   Jtv(j) = int_0^{t_n} Sigma^R(t_n,s) G^](s,tau_j) ds
 *          + int_0^beta Sigma^](t_n,tb) G^M(tb - tau_j) dtb   (Eq. KBE3)
 * The Matsubara convolution is split at tb = tau_j because G^M jumps there:
 * on [0, tau_j] the argument is negative and antiperiodicity gives
 * G^M(tb - tau_j) = -G^M(tb - tau_j + beta); on [tau_j, beta] it is
 * G^M(tb - tau_j) directly.  Each piece is integrated with its own rule.
 * Jtv is computed for j in [j0, j1) (stored from Jtv[0]). */
void orc_collision(int N, int nt, int ntau, int64_t ldt, const cplx *kp, const cplx *rdiag,
                   const cplx *tv, const cplx *mat, const cplx *ret, const cplx *les,
                   const cplx *stv, const double *w, const double *wfull, const double *wf,
                   const double *wb, int n, int m0, int m1, int j0, int j1, int flags, cplx *IR,
                   cplx *IL, cplx *Itv, cplx *Jtv) {
  green g = {N, nt, ntau, ldt, kp, rdiag, tv, mat};
  int64_t bs = (int64_t)N * N;
#pragma omp parallel for schedule(dynamic, 1)
  for (int m = m0; m < m1; ++m) {
    cplx blk[256];
    if (flags & F_IR) {
      cplx *o = IR + (m - m0) * bs;
      memset(o, 0, sizeof(cplx) * bs);
      for (int s = 0; s <= n; ++s) {
        if (flags & F_GREATER) get_gtr(&g, s, m, blk);
        else get_les(&g, s, m, blk);
        mm_acc(N, o, w[(int64_t)n * nt + s], ret + s * bs, blk, 0);
      }
    }
    if (flags & F_IL) {
      cplx *o = IL + (m - m0) * bs;
      cplx sg[256];
      memset(o, 0, sizeof(cplx) * bs);
      for (int s = 0; s <= m; ++s) {
        get_ret(&g, m, s, blk);
        const cplx *sx = les + s * bs;
        if (flags & F_GREATER) { /* Sigma^>(t_n,t_s) = Sigma^R + Sigma^< for s <= n */
          for (int e = 0; e < bs; ++e) sg[e] = ret[s * bs + e] + les[s * bs + e];
          sx = sg;
        }
        mm_acc(N, o, w[(int64_t)m * nt + s], sx, blk, 1);
      }
    }
    if ((flags & F_ITV) && ntau > 0) {
      cplx *o = Itv + (m - m0) * bs;
      memset(o, 0, sizeof(cplx) * bs);
      for (int j = 0; j < ntau; ++j) {
        const cplx *x = tv + ((int64_t)m * ntau + tau_mirror(ntau, j)) * bs;
        mm_acc(N, o, -I * wfull[j], stv + j * bs, x, 1);
      }
    }
  }
  if ((flags & F_JTV) && ntau > 0) {
    int J = ntau - 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = j0; j < j1; ++j) {
      cplx *o = Jtv + (j - j0) * bs;
      memset(o, 0, sizeof(cplx) * bs);
      for (int s = 0; s <= n; ++s)
        mm_acc(N, o, w[(int64_t)n * nt + s], ret + s * bs, tv + ((int64_t)s * ntau + j) * bs, 0);
      /* piece on [0, tau_j]: G^M(tau_l - tau_j) = -G^M(beta + tau_l - tau_j) */
      for (int l = 0; l <= j; ++l)
        mm_acc(N, o, -wf[(int64_t)j * ntau + l], stv + l * bs, mat + (J + l - j) * bs, 0);
      /* piece on [tau_j, beta]: G^M(tau_l - tau_j) with a non-negative argument */
      for (int l = j; l < ntau; ++l)
        mm_acc(N, o, wb[(int64_t)j * ntau + l], stv + l * bs, mat + (l - j) * bs, 0);
    }
  }
}

/* The integrals of orc_collision (IR, IL, Itv) at one point (t_n, t_m), from the
 * blocks that row reads (its "cross"): col[s] = kp[s][m] for s <= m, row[s] =
 * kp[m][s] for s <= n, rdg = G^R(t_m,t_m), tvm[j] = G^](t_m,tau_j); weight rows
 * wn = w[n][.] and wm = w[m][.]; wfull the full-range tau rule.  By the lesser
 * symmetry G^<(t_s,t_m) = col[s] for s <= m and -row[s]^dagger for s > m; G^R(t_m,t_s)
 * is row[s] for s < m and rdg at s = m.  Same sums, same order as orc_collision. */
void orc_collision_row(int N, int ntau, int n, int m, const cplx *ret, const cplx *les,
                       const cplx *stv, const cplx *col, const cplx *row, const cplx *rdg,
                       const cplx *tvm, const double *wn, const double *wm, const double *wfull,
                       int flags, cplx *IR, cplx *IL, cplx *Itv) {
  int64_t bs = (int64_t)N * N;
  cplx blk[256];
  if (flags & F_IR) {
    memset(IR, 0, sizeof(cplx) * bs);
    for (int s = 0; s <= n; ++s) {
      if (s <= m) {
        memcpy(blk, col + s * bs, sizeof(cplx) * bs);
      } else {
        const cplx *x = row + s * bs;
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j) blk[i * N + j] = -conj(x[j * N + i]);
      }
      mm_acc(N, IR, wn[s], ret + s * bs, blk, 0);
    }
  }
  if (flags & F_IL) {
    memset(IL, 0, sizeof(cplx) * bs);
    for (int s = 0; s <= m; ++s) mm_acc(N, IL, wm[s], les + s * bs, s < m ? row + s * bs : rdg, 1);
  }
  if (flags & F_ITV) {
    memset(Itv, 0, sizeof(cplx) * bs);
    for (int j = 0; j < ntau; ++j)
      mm_acc(N, Itv, -I * wfull[j], stv + j * bs, tvm + tau_mirror(ntau, j) * bs, 1);
  }
}

/* ------------------------------------------------------------------------- */
/* Adjoint (vector-Jacobian product) of orc_collision.  Complex gradients     */
/* follow PyTorch's convention: for real loss L and complex z the gradient is */
/* dL/dRe z + i dL/dIm z.  For C = c A op(B):                                 */
/*   op = identity: gA = conj(c) gC B^dagger,  gB = conj(c) A^dagger gC       */
/*   op = dagger  : gA = conj(c) gC B,         gB = c gC^dagger A             */
/* Storage entries are independent variables, so the gradient of a value      */
/* read through G^< = -(stored)^dagger is -(gradient)^dagger.                 */
/* Self-energy gradients are overwritten; Green's-function gradients are      */
/* accumulated.                                                               */
/* ------------------------------------------------------------------------- */

static void add_les_grad(const green *g, cplx *gkp, int a, int b, const cplx *gval) {
  /* gval is the gradient with respect to G^<(t_a,t_b) */
  int N = g->N;
  if (a <= b) {
    cplx *x = gkp + ((int64_t)a * g->ldt + b) * N * N;
    for (int e = 0; e < N * N; ++e) x[e] += gval[e];
  } else {
    cplx *x = gkp + ((int64_t)b * g->ldt + a) * N * N;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) x[j * N + i] += -conj(gval[i * N + j]);
  }
}

void orc_collision_vjp(int N, int nt, int ntau, int64_t ldt, const cplx *kp, const cplx *rdiag,
                       const cplx *tv, const cplx *mat, const cplx *ret, const cplx *les,
                       const cplx *stv, const double *w, const double *wfull, const double *wf,
                       const double *wb, int n, int m0, int m1, int flags, const cplx *gIR,
                       const cplx *gIL, const cplx *gItv, const cplx *gJtv, cplx *gkp,
                       cplx *grdiag, cplx *gtv, cplx *gmat, cplx *gret, cplx *gles, cplx *gstv) {
  green g = {N, nt, ntau, ldt, kp, rdiag, tv, mat};
  int64_t bs = (int64_t)N * N;
  int J = ntau - 1;
  memset(gret, 0, sizeof(cplx) * bs * (n + 1));
  memset(gles, 0, sizeof(cplx) * bs * (n + 1));
  if (ntau > 0) memset(gstv, 0, sizeof(cplx) * bs * ntau);
  cplx blk[256], tmp[256];
  /* Gradients of the self-energy row: one pass over the same terms as the
   * forward, each term's adjoint on its self-energy factor. */
  for (int m = m0; m < m1; ++m) {
    if (flags & F_IR)
      for (int s = 0; s <= n; ++s) {
        /* IR term: w[n][s] ret[s] G^<(s,m)  (greater form: G^>(s,m)) */
        if (flags & F_GREATER) get_gtr(&g, s, m, blk);
        else get_les(&g, s, m, blk);
        mm_acc(N, gret + s * bs, w[(int64_t)n * nt + s], gIR + (m - m0) * bs, blk, 1);
      }
    if (flags & F_IL)
      for (int s = 0; s <= m; ++s) {
        get_ret(&g, m, s, blk); /* IL term: w[m][s] les[s] G^R(m,s)^dagger */
        mm_acc(N, gles + s * bs, w[(int64_t)m * nt + s], gIL + (m - m0) * bs, blk, 0);
        /* greater form: the factor is Sigma^> = ret + les, so ret gets the same gradient */
        if (flags & F_GREATER)
          mm_acc(N, gret + s * bs, w[(int64_t)m * nt + s], gIL + (m - m0) * bs, blk, 0);
      }
    if ((flags & F_ITV) && ntau > 0)
      for (int j = 0; j < ntau; ++j) { /* Itv term: (-i wfull[j]) stv[j] tv[m][J-j]^dagger */
        const cplx *x = tv + ((int64_t)m * ntau + tau_mirror(ntau, j)) * bs;
        mm_acc(N, gstv + j * bs, conj(-I * wfull[j]), gItv + (m - m0) * bs, x, 0);
      }
  }
  if ((flags & F_JTV) && ntau > 0)
    for (int j = 0; j < ntau; ++j) {
      for (int s = 0; s <= n; ++s) /* Jtv term: w[n][s] ret[s] tv[s][j] */
        mm_acc(N, gret + s * bs, w[(int64_t)n * nt + s], gJtv + j * bs,
               tv + ((int64_t)s * ntau + j) * bs, 1);
      for (int l = 0; l <= j; ++l) /* -wf[j][l] stv[l] mat[J+l-j] */
        mm_acc(N, gstv + l * bs, -wf[(int64_t)j * ntau + l], gJtv + j * bs, mat + (J + l - j) * bs, 1);
      for (int l = j; l < ntau; ++l) /* wb[j][l] stv[l] mat[l-j] */
        mm_acc(N, gstv + l * bs, wb[(int64_t)j * ntau + l], gJtv + j * bs, mat + (l - j) * bs, 1);
    }
  /* Gradients of the Green's function: the adjoint on the other factor. */
  for (int m = m0; m < m1; ++m) {
    if (flags & F_IR)
      for (int s = 0; s <= n; ++s) { /* gB = conj(c) A^dagger gC for B = G^<(s,m) */
        memset(tmp, 0, sizeof(cplx) * bs);
        mm_acc_hn(N, tmp, w[(int64_t)n * nt + s], ret + s * bs, gIR + (m - m0) * bs);
        add_les_grad(&g, gkp, s, m, tmp);
        if (flags & F_GREATER) {
          /* B = G^>(s,m) = G^<(s,m) + D(s,m): D = G^R(s,m) stored at kp[s][m] (s > m), at
           * rdiag[m] (s = m), and D = -G^R(m,s)^dagger with G^R(m,s) at kp[m][s] (s < m) */
          if (s > m) {
            cplx *x = gkp + ((int64_t)s * ldt + m) * bs;
            for (int e = 0; e < bs; ++e) x[e] += tmp[e];
          } else if (s == m) {
            cplx *x = grdiag + (int64_t)m * bs;
            for (int e = 0; e < bs; ++e) x[e] += tmp[e];
          } else {
            cplx *x = gkp + ((int64_t)m * ldt + s) * bs;
            for (int i = 0; i < N; ++i)
              for (int j = 0; j < N; ++j) x[j * N + i] += -conj(tmp[i * N + j]);
          }
        }
      }
    if (flags & F_IL)
      for (int s = 0; s <= m; ++s) { /* B = G^R(m,s) used as B^dagger: gB = c gC^dagger A */
        cplx sg[256];
        const cplx *sa = les + s * bs;
        if (flags & F_GREATER) { /* A = Sigma^>(t_n,t_s) = ret + les */
          for (int e = 0; e < bs; ++e) sg[e] = ret[s * bs + e] + les[s * bs + e];
          sa = sg;
        }
        memset(tmp, 0, sizeof(cplx) * bs);
        mm_acc_hn(N, tmp, w[(int64_t)m * nt + s], gIL + (m - m0) * bs, sa);
        cplx *x = (s == m) ? grdiag + (int64_t)m * bs : gkp + ((int64_t)m * ldt + s) * bs;
        for (int e = 0; e < bs; ++e) x[e] += tmp[e];
      }
    if ((flags & F_ITV) && ntau > 0)
      for (int j = 0; j < ntau; ++j) {
        memset(tmp, 0, sizeof(cplx) * bs);
        mm_acc_hn(N, tmp, -I * wfull[j], gItv + (m - m0) * bs, stv + j * bs);
        cplx *x = gtv + ((int64_t)m * ntau + tau_mirror(ntau, j)) * bs;
        for (int e = 0; e < bs; ++e) x[e] += tmp[e];
      }
  }
  if ((flags & F_JTV) && ntau > 0)
    for (int j = 0; j < ntau; ++j) {
      for (int s = 0; s <= n; ++s) {
        memset(tmp, 0, sizeof(cplx) * bs);
        mm_acc_hn(N, tmp, w[(int64_t)n * nt + s], ret + s * bs, gJtv + j * bs);
        cplx *x = gtv + ((int64_t)s * ntau + j) * bs;
        for (int e = 0; e < bs; ++e) x[e] += tmp[e];
      }
      for (int l = 0; l <= j; ++l) {
        memset(tmp, 0, sizeof(cplx) * bs);
        mm_acc_hn(N, tmp, -wf[(int64_t)j * ntau + l], stv + l * bs, gJtv + j * bs);
        cplx *x = gmat + (int64_t)(J + l - j) * bs;
        for (int e = 0; e < bs; ++e) x[e] += tmp[e];
      }
      for (int l = j; l < ntau; ++l) {
        memset(tmp, 0, sizeof(cplx) * bs);
        mm_acc_hn(N, tmp, wb[(int64_t)j * ntau + l], stv + l * bs, gJtv + j * bs);
        cplx *x = gmat + (int64_t)(l - j) * bs;
        for (int e = 0; e < bs; ++e) x[e] += tmp[e];
      }
    }
}

/* ------------------------------------------------------------------------- */
/* Adjoint of orc_sigma_row.  Sigma^<_ij(n,s) = U L^2 Gt, Sigma^>_ij(n,s) =   */
/* U Gg^2 Lt with U = u_i u_j, L = G^<_ij(n,s), Gt = G^>_ji(s,n),             */
/* Gg = G^>_ij(n,s), Lt = G^<_ji(s,n); Sigma^R = Sigma^> - Sigma^<.  Each      */
/* factor is holomorphic in the value it reads, so its gradient is             */
/* gW * conj(dW/dz); the values are then traced back through the storage     */
/* accessors (a value read as -conj(stored) sends back -conj(gradient)).      */
/* The interaction is real: gu_k += Re(conj(gW) dW/du_k).  Gradients are      */
/* accumulated.                                                               */
/* ------------------------------------------------------------------------- */

/* gradient with respect to G^<_ij(t_a,t_b) for a single element */
static void les_elem_grad(const green *g, cplx *gkp, int a, int b, int i, int j, cplx gv) {
  int N = g->N;
  if (a <= b) gkp[((int64_t)a * g->ldt + b) * N * N + i * N + j] += gv;
  else gkp[((int64_t)b * g->ldt + a) * N * N + j * N + i] += -conj(gv);
}

static void ret_elem_grad(const green *g, cplx *gkp, cplx *grdiag, int a, int b, int i, int j,
                          cplx gv) {
  int N = g->N;
  if (a == b) grdiag[(int64_t)a * N * N + i * N + j] += gv;
  else gkp[((int64_t)a * g->ldt + b) * N * N + i * N + j] += gv;
}

/* gradient with respect to G^>_ij(t_a,t_b) */
static void gtr_elem_grad(const green *g, cplx *gkp, cplx *grdiag, int a, int b, int i, int j,
                          cplx gv) {
  if (a >= b) {
    ret_elem_grad(g, gkp, grdiag, a, b, i, j, gv);
    les_elem_grad(g, gkp, a, b, i, j, gv);
  } else {
    gtr_elem_grad(g, gkp, grdiag, b, a, j, i, -conj(gv));
  }
}

void orc_sigma_row_vjp(int N, int nt, int ntau, int64_t ldt, const cplx *kp, const cplx *rdiag,
                       const cplx *tv, const double *u, int n, const cplx *gret, const cplx *gles,
                       const cplx *gstv, cplx *gkp, cplx *grdiag, cplx *gtv, double *gu) {
  green g = {N, nt, ntau, ldt, kp, rdiag, tv, NULL};
  int64_t bs = (int64_t)N * N;
  for (int s = 0; s <= n; ++s) {
    cplx lns[256], lsn[256], gns[256], gsn[256];
    get_les(&g, n, s, lns);
    get_les(&g, s, n, lsn);
    get_gtr(&g, n, s, gns);
    get_gtr(&g, s, n, gsn);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        double U = u[i] * u[j];
        cplx L = lns[i * N + j], Gt = gsn[j * N + i], Gg = gns[i * N + j], Lt = lsn[j * N + i];
        cplx gR = gret[s * bs + i * N + j], gL = gles[s * bs + i * N + j];
        cplx g_gtr = gR;      /* Sigma^> enters Sigma^R with + */
        cplx g_les = gL - gR; /* Sigma^< enters Sigma^< with + and Sigma^R with - */
        cplx dL = g_les * conj(2.0 * U * L * Gt);
        cplx dGt = g_les * conj(U * L * L);
        cplx dGg = g_gtr * conj(2.0 * U * Gg * Lt);
        cplx dLt = g_gtr * conj(U * Gg * Gg);
        les_elem_grad(&g, gkp, n, s, i, j, dL);
        gtr_elem_grad(&g, gkp, grdiag, s, n, j, i, dGt);
        gtr_elem_grad(&g, gkp, grdiag, n, s, i, j, dGg);
        les_elem_grad(&g, gkp, s, n, j, i, dLt);
        double cu = creal(conj(g_les) * (L * L * Gt)) + creal(conj(g_gtr) * (Gg * Gg * Lt));
        gu[i] += u[j] * cu;
        gu[j] += u[i] * cu;
      }
  }
  int J = ntau - 1;
  for (int l = 0; l < ntau; ++l)
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        double U = u[i] * u[j];
        cplx x = tv[((int64_t)n * ntau + l) * bs + i * N + j];
        cplx y = tv[((int64_t)n * ntau + (J - l)) * bs + i * N + j];
        cplx gs = gstv[(int64_t)l * bs + i * N + j];
        /* W = U x^2 conj(y): holomorphic in x, antiholomorphic in y */
        gtv[((int64_t)n * ntau + l) * bs + i * N + j] += gs * conj(2.0 * U * x * conj(y));
        gtv[((int64_t)n * ntau + (J - l)) * bs + i * N + j] += conj(gs) * (U * x * x);
        double cu = creal(conj(gs) * (x * x * conj(y)));
        gu[i] += u[j] * cu;
        gu[j] += u[i] * cu;
      }
}

/* ------------------------------------------------------------------------- */
/* Second-Born self-energy with a general four-index interaction (Eq. SE), at  */
/* one pair of time arguments:                                                */
/*   out_ij = sum_{f,d,e,a,b,c} U_ifde Uex_jabc A_fb A_ea C_cd,               */
/*   Uex_jabc = 2 U_jbac - U_jabc,                                            */
/* with A = G^<>(t,t') and C = G^><(t',t) (or the mixed-branch pair).  U is   */
/* real, U[i][f][d][e] = U_ifde.  Six nested sums per output entry, in the    */
/* printed order of the indices; OpenMP over the output entries only.         */
/* ------------------------------------------------------------------------- */
void orc_gf2_block(int N, const double *U, const cplx *A, const cplx *C, cplx *out) {
#define U4(i, f, d, e) U[(((int64_t)(i) * N + (f)) * N + (d)) * N + (e)]
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      cplx acc = 0.0;
      for (int f = 0; f < N; ++f)
        for (int d = 0; d < N; ++d)
          for (int e = 0; e < N; ++e)
            for (int a = 0; a < N; ++a)
              for (int b = 0; b < N; ++b)
                for (int c = 0; c < N; ++c) {
                  double ex = 2.0 * U4(j, b, a, c) - U4(j, a, b, c);
                  acc += U4(i, f, d, e) * ex * A[f * N + b] * A[e * N + a] * C[c * N + d];
                }
      out[i * N + j] = acc;
    }
#undef U4
}

/* Thread count of the OpenMP loops above (timing of the oracle as a CPU baseline; the results
 * do not depend on it: every output is summed by one thread in a fixed order). */
void orc_set_threads(int k) {
#ifdef _OPENMP
  omp_set_num_threads(k);
#else
  (void)k;
#endif
}

