/*
 * kbe.h — C ABI of the MI355X history-integral library (libkbe.so).
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950) in FP64, the
 * data-parallel hot path of adaptive Kadanoff-Baym propagation as described in
 * T. Blommel, D. J. Gardner, C. S. Woodward, E. Gull, "Adaptive Time Stepping
 * for the Two-Time Integro-Differential Kadanoff-Baym Equations",
 * arXiv:2405.08737:
 *   - the composite quadrature weights of Sec. "Adaptive History Integration"
 *     (Eq. weights and the weight-row recursion),
 *   - the second-Born (GF2) self-energy of Eq. SE for a local interaction,
 *   - the history integrals of Eq. KBE2 (lesser form) and Eq. KBE3,
 *   - and the adjoints (vector-Jacobian products) of the last two.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Numbers.  kbe_c128 is complex128: {re, im} doubles, the layout of C99
 * double complex and of torch.complex128.  N x N blocks are row-major.
 *
 * Storage of a Keldysh function (struct kbe_green), all device memory:
 *   kp    [nt rows][ldt][N][N]  kp[a][b] = G^<(t_a,t_b) for a <= b (upper
 *                               triangle and diagonal), G^R(t_a,t_b) for a > b.
 *                               The paper stores one side of the diagonal per
 *                               component (Sec. "Implementation"); the retarded
 *                               value below it is G^> - G^< there.
 *   rdiag [nt][N][N]            G^R(t_a,t_a) (the equal-time retarded value;
 *                               -i*1 for a physical G).
 *   tv    [nt][ntau][N][N]      G^](t_m,tau_j), the mixed component.
 *   mat   [ntau][N][N]          G^M(tau_j); mat[0] = G^M(0+), mat[ntau-1] = G^M(beta-).
 * Values at other arguments follow from the symmetries of Sec. "Kadanoff Baym
 * Equations": G^<(t,t') = -G^<(t',t)^dagger, G^>(t,t') = G^R + G^< for t >= t',
 * G^>(t,t') = -G^>(t',t)^dagger, G^[(tau,t) = G^](t,beta-tau)^dagger.
 * Every array entry is an independent variable (gradients are not tied across
 * mirrored entries).
 *
 * Imaginary time.  tau_j = j*beta/(ntau-1) (a uniform, symmetric grid, so
 * beta - tau_j = tau_{ntau-1-j}); ntau = 0 removes the thermal branch
 * (Eq. KBE3 and the tau integrals are dropped, as the paper allows).
 *
 * Self-energy row at t_n (struct kbe_sigma_row), device memory:
 *   ret [n+1][N][N]  Sigma^R(t_n,t_s), s = 0..n (s = n: the one-sided limit)
 *   les [n+1][N][N]  Sigma^<(t_n,t_s)
 *   tv  [ntau][N][N] Sigma^](t_n,tau_j)
 *
 * Ownership.  The caller owns every buffer.  The library allocates no device
 * memory: scratch memory is a caller-supplied device workspace whose size the
 * matching *_workspace() query returns (its parts start at 256-byte offsets:
 * pass it 256-byte aligned, as hipMalloc returns it).  The one exception is the
 * fixed scratch array behind kbe_collision_noalloc (KBE_NOALLOC_SCRATCH_BYTES
 * per device, part of the library's device code, held until the process
 * ends).  kbe_propagate_adaptive holds 4 KiB of page-locked host memory for the
 * duration of the call (the error norms its controller reads).
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  All device
 * work is enqueued asynchronously on it; no entry point synchronises the host
 * except kbe_weights, which reads host arrays before returning, and the two
 * iterations driven from the host: kbe_propagate_adaptive (error norms at
 * every fixed-point iteration) and kbe_equilibrium (the change once per
 * iteration).
 *
 * Errors.  Every entry point validates its arguments on the host before
 * enqueuing anything and returns a kbe_status; on an error nothing has been
 * enqueued and kbe_last_error() (thread-local) describes the problem.  A HIP
 * launch failure returns KBE_EHIP.  Results are deterministic: no floating-
 * point atomics are used, so repeated calls give bitwise-identical results.
 */
#ifndef KBE_H
#define KBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double re, im;
} kbe_c128;

typedef enum {
  KBE_OK = 0,
  KBE_EINVAL = 1,  /* NULL pointer, bad size, inconsistent shapes, bad grid */
  KBE_ERANGE = 2,  /* n, m-range or order outside the allowed range */
  KBE_ENOMEM = 3,  /* workspace smaller than the *_workspace() query */
  KBE_EHIP = 4,    /* a HIP runtime call or kernel launch failed */
  KBE_ENOTSUP = 5, /* valid request this build does not support */
  KBE_ESTEP = 6    /* the adaptive controller could not reach t_end (step size underflow or the
                      grid capacity exhausted); the trace holds the steps accepted until then */,
  KBE_ECONV = 7    /* kbe_equilibrium did not converge within its iteration limit (or the
                      iteration diverged); the output holds the last iterate */
} kbe_status;

#define KBE_NMAX 16 /* largest orbital count N */
#define KBE_KMAX 20 /* largest quadrature order (nodes per interval) */

/* Output selection for kbe_collision / kbe_collision_vjp. */
#define KBE_OUT_IR 0x1u  /* retarded integral   I^R(t_n,t_m) */
#define KBE_OUT_IL 0x2u  /* lesser integral     I^<(t_n,t_m) */
#define KBE_OUT_ITV 0x4u /* tau integral        I^](t_n,t_m) (mixing term of Eq. KBE2) */
#define KBE_OUT_JTV 0x8u /* left-mixing RHS     J^](t_n,tau_j) (history terms of Eq. KBE3) */
#define KBE_OUT_ALL 0xFu
/* Execution switches. */
#define KBE_FORCE_GENERIC 0x100u  /* use the vector-ALU kernels even where matrix-core (MFMA)
                                     kernels exist (N = 16); results agree to rounding */
#define KBE_GRAD_OVERWRITE 0x200u /* VJP: overwrite the Green's-function gradient blocks the
                                     forward call reads instead of adding to them */
#define KBE_GREATER 0x400u        /* kbe_collision: the greater form of Eq. KBE2 (the paper's
                                     choice below the diagonal): I^R with G^>(t_s,t_m) in place
                                     of G^<(t_s,t_m), assembled from both triangles, and I^< with
                                     Sigma^> = Sigma^R + Sigma^< (from the same self-energy row)
                                     in place of Sigma^<; I^] and J^] are the same in both forms.
                                     Supported by kbe_collision and its adjoint
                                     kbe_collision_vjp (whose gradients then also reach G^R
                                     through G^> and Sigma^R through Sigma^>), on the same kernels
                                     as the lesser form plus extra term classes.  The batch calls
                                     reject it (KBE_EINVAL). */

/* One Keldysh function on the grid (G, or a gradient with the same shape). */
typedef struct {
  int32_t N;       /* orbitals, 1..KBE_NMAX */
  int32_t nt;      /* real-time points stored, >= 1 */
  int32_t ntau;    /* imaginary-time points: 0 or >= 2 */
  int64_t ldt;     /* row stride of kp in blocks, >= nt */
  kbe_c128 *kp;    /* device [nt][ldt][N][N] */
  kbe_c128 *rdiag; /* device [nt][N][N] */
  kbe_c128 *tv;    /* device [nt][ntau][N][N] (may be NULL when ntau == 0) */
  kbe_c128 *mat;   /* device [ntau][N][N]     (may be NULL when ntau == 0) */
} kbe_green;

typedef struct {
  kbe_c128 *ret; /* device [n+1][N][N] */
  kbe_c128 *les; /* device [n+1][N][N] */
  kbe_c128 *tv;  /* device [ntau][N][N] (may be NULL when ntau == 0) */
} kbe_sigma_row;

/* Time grid (host memory). */
typedef struct {
  int32_t nt;           /* points, >= 1 */
  const double *t;      /* host [nt]: t[0] = 0 < t[1] < ... (the grid starts at 0, Sec. KBE) */
  const int32_t *order; /* host [nt]: nodes of the interpolant on interval p (p >= 1),
                           1..KBE_KMAX; order[0] is ignored */
  int32_t ntau;         /* 0 or >= 2 */
  double beta;          /* inverse temperature, > 0 when ntau > 0 */
  int32_t tau_order;    /* nodes per tau interval, 1..KBE_KMAX (ignored when ntau == 0) */
} kbe_grid;

/* Quadrature weights (device memory), as produced by kbe_weights. */
typedef struct {
  const double *w;        /* [nt][nt]: w[n][s], integral over [0, t_n] */
  const double *wtau;     /* [ntau]: integral over [0, beta] */
  const double *wtau_fwd; /* [ntau][ntau]: wtau_fwd[j][l], integral over [0, tau_j] */
} kbe_wts;

/* ---------------------------------------------------------------------------
 * kbe_weights — quadrature weights (Sec. "Adaptive History Integration",
 * Eq. weights and the row recursion that follows it).
 *
 * Real time: interval p = [t_{p-1}, t_p] is integrated with the Lagrange
 * interpolant through its k_p = min(order[p], p+1) most recent nodes
 * t_{p-k_p+1..p}; the local weights solve the moment equations of Eq. weights
 * (LU with full pivoting, as in the paper, but written in a Legendre basis on
 * the window instead of monomials, which keeps order 20 well conditioned),
 * and row n of w is row n-1 plus the local weights of interval n
 * (so w[n][s] = 0 for s > n and row 0 is 0).  "order" counts nodes: order 2 is
 * the trapezoid rule, order k is exact for polynomials of degree < k.
 * Imaginary time (ntau > 0): wtau_fwd[j] integrates over [0, tau_j] using
 * min(tau_order, j+1) nodes per interval on windows kept inside [0, tau_j];
 * wtau[l] = (wtau_fwd[J][l] + wtau_fwd[J][J-l]) / 2 integrates over [0, beta]
 * and is symmetric (the paper's DLR tau basis is replaced by this rule).
 *
 * Arguments: g (host) describes the grid; w [nt][nt], wtau [ntau] and
 * wtau_fwd [ntau][ntau] are device outputs (the tau ones may be NULL when
 * ntau == 0); ws is a device workspace of at least kbe_weights_workspace(g)
 * bytes.  The host arrays may be released when the call returns.
 * Errors: KBE_EINVAL for NULL pointers, nt < 1, t[0] != 0, t not strictly
 * increasing, ntau == 1, beta <= 0; KBE_ERANGE for an order outside
 * 1..KBE_KMAX; KBE_ENOMEM for a short workspace; KBE_ENOTSUP when `stream` is
 * being captured into a HIP graph (the call copies host memory: use
 * kbe_weights_dev there).
 * ------------------------------------------------------------------------- */
size_t kbe_weights_workspace(const kbe_grid *g);
kbe_status kbe_weights(const kbe_grid *g, double *w, double *wtau, double *wtau_fwd, void *ws,
                       size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_weights_dev — kbe_weights for a grid already in device memory: the same
 * weights, with no host copy and no synchronisation, so the call can be
 * captured in a HIP graph (with the calls that use the weights).
 *
 * Arguments: t device [nt], order device [nt] (as in kbe_grid); ntau, beta,
 * tau_order as in kbe_grid; w, wtau, wtau_fwd device outputs as for
 * kbe_weights; status: optional device int32 (NULL: no check) that receives 0
 * for a valid grid, KBE_EINVAL if t[0] != 0 or t is not strictly increasing,
 * KBE_ERANGE for an order outside 1..KBE_KMAX (the weights of such a grid are
 * computed with the orders clamped into range and are not meaningful); ws a
 * device workspace of kbe_weights_dev_workspace(nt, ntau) bytes.
 * Errors (returned, nothing enqueued): KBE_EINVAL for NULL pointers, nt < 1,
 * ntau == 1, beta <= 0 with ntau > 0; KBE_ERANGE for tau_order outside
 * 1..KBE_KMAX; KBE_ENOMEM for a short workspace.
 * ------------------------------------------------------------------------- */
size_t kbe_weights_dev_workspace(int32_t nt, int32_t ntau);
kbe_status kbe_weights_dev(const double *t, const int32_t *order, int32_t nt, int32_t ntau,
                           double beta, int32_t tau_order, double *w, double *wtau,
                           double *wtau_fwd, int32_t *status, void *ws, size_t ws_bytes,
                           void *stream);

/* ---------------------------------------------------------------------------
 * kbe_step_weights — the local weights of Eq. weights for every interval and
 * every node count: lam[p][k-1][i] (i < k) integrates over [t_{p-1}, t_p] the
 * Lagrange interpolant through the k nodes t_{p-k+1..p}, for
 * k = 1..min(order[p], p+1); other entries (and row p = 0) are zero.  With
 * k = min(order[p], p+1) these are the local weights that the history rows of
 * kbe_weights add up; smaller k are the rules kbe_propagate uses for elements
 * whose history begins inside the window.
 *
 * Arguments: t, order device [nt]; lam device [nt][KBE_KMAX][KBE_KMAX];
 * status optional, as for kbe_weights_dev.  No workspace.  Capturable.
 * Errors: KBE_EINVAL for NULL pointers or nt < 1.
 * ------------------------------------------------------------------------- */
kbe_status kbe_step_weights(const double *t, const int32_t *order, int32_t nt, double *lam,
                            int32_t *status, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_sigma_2b — second-Born self-energy row at t_n (Eq. SE).
 *
 * For a local interaction U_{ijkl} = u_i d_ij d_jk d_kl the exchange tensor is
 * U^Ex_{jjjj} = u_j and Eq. SE reduces to
 *   Sigma^<_ij(t,t') = u_i u_j G^<_ij(t,t')^2 G^>_ji(t',t)
 *   Sigma^>_ij(t,t') = u_i u_j G^>_ij(t,t')^2 G^<_ji(t',t)
 *   Sigma^]_ij(t,tau) = u_i u_j G^]_ij(t,tau)^2 G^[_ji(tau,t)
 * evaluated for t = t_n, t' = t_s (s = 0..n) and all tau_j.  Outputs:
 * out->ret[s] = Sigma^>(t_n,t_s) - Sigma^<(t_n,t_s) (= Sigma^R for s < n, its
 * one-sided limit at s = n), out->les[s] = Sigma^<(t_n,t_s), out->tv[j].
 * G values are read through the storage symmetries stated above: row n and
 * column n of kp, rdiag[n] and tv[n].
 *
 * Arguments: G (device arrays); u device [N] (a scalar U fills all entries);
 * 0 <= n < G->nt; out device arrays (overwritten).
 * Errors: KBE_EINVAL (NULL, bad shape), KBE_ERANGE (n).
 * ------------------------------------------------------------------------- */
kbe_status kbe_sigma_2b(const kbe_green *G, const double *u, int32_t n, const kbe_sigma_row *out,
                        void *stream);

/* ---------------------------------------------------------------------------
 * kbe_sigma_2b_full — the second-Born self-energy of kbe_sigma_2b (local U,
 * Eq. SE) for every time pair, in the KP storage of G ("full mode", for tests
 * and for callers that want the whole Sigma rather than one row):
 *   S->kp[a][b] = Sigma^<(t_a,t_b) (a <= b),  Sigma^>(t_a,t_b) - Sigma^<(t_a,t_b) (a > b)
 *   S->rdiag[a] = Sigma^>(t_a,t_a) - Sigma^<(t_a,t_a)   (the one-sided Sigma^R(t,t))
 *   S->tv[a][l] = Sigma^](t_a,tau_l)
 * for a, b < G->nt; every value from the formula at its own arguments (no
 * symmetry of Sigma is assumed).  S->mat is not written (Eq. SE gives no
 * Matsubara component).
 *
 * Arguments: G and S device arrays with the same N, nt and ntau (S->ldt >= nt
 * may differ from G's); u device [N].  Errors: KBE_EINVAL (NULL, shapes).
 * ------------------------------------------------------------------------- */
kbe_status kbe_sigma_2b_full(const kbe_green *G, const double *u, const kbe_green *S,
                             void *stream);

/* ---------------------------------------------------------------------------
 * kbe_sigma_2b_batch — the rows of kbe_sigma_2b for many systems in one launch
 * (a project addition, the self-energy stage of batched history rows): item i
 * is row n of its own system (its own N, grid, storage and u), with the same
 * formulas and element code as kbe_sigma_2b, so each row equals that call's bit
 * for bit.
 *
 * items: host array of count items (validated here); items_dev: the same array
 * in device memory (what the kernel reads; it must equal items when the work
 * runs).  Nothing is copied from host memory and nothing is allocated, so the
 * call can be captured in a HIP graph (with the kbe_collision_batch call that
 * reads the rows).  Errors: KBE_EINVAL (NULL pointers, N, nt, ntau or ldt out
 * of range), KBE_ERANGE (n outside [0, nt), count outside [0, KBE_BATCH_MAX]).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t N;                        /* orbitals, 1..KBE_NMAX */
  int32_t nt;                       /* real-time points of the system's storage, >= 1 */
  int32_t ntau;                     /* imaginary-time points: 0 or >= 2 */
  int32_t n;                        /* the row, 0 <= n < nt */
  int64_t ldt;                      /* kp row stride in blocks, >= nt */
  const kbe_c128 *kp, *rdiag, *tv;  /* the system's G, as in kbe_green (tv NULL if ntau == 0) */
  const double *u;                  /* [N] local interaction */
  kbe_c128 *ret, *les, *stv;        /* out: [n+1], [n+1], [ntau] (stv NULL if ntau == 0) */
} kbe_sigma_batch_item;

kbe_status kbe_sigma_2b_batch(const kbe_sigma_batch_item *items,
                              const kbe_sigma_batch_item *items_dev, int32_t count, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_sigma_gf2 — second-Born self-energy row at t_n with a general
 * four-index interaction (Eq. SE):
 *   Sigma^<>_ij(t,t') = sum U_ifde Uex_jabc G^<>_fb(t,t') G^<>_ea(t,t') G^><_cd(t',t)
 *   Sigma^]_ij(t,tau) = sum U_ifde Uex_jabc G^]_fb(t,tau) G^]_ea(t,tau) G^[_cd(tau,t)
 * summed over f, d, e, a, b, c, with Uex_jabc = 2 U_jbac - U_jabc and
 * G^[(tau,t) = G^](t,beta-tau)^dagger, for t = t_n, t' = t_s (s = 0..n) and
 * every tau_l.  Outputs as kbe_sigma_2b: out->ret[s] = Sigma^> - Sigma^<,
 * out->les[s] = Sigma^<, out->tv[l].  With U_ijkl = u_i d_ij d_jk d_kl the
 * result is kbe_sigma_2b's.  Cost: 4 N^5 complex multiply-adds per block.
 *
 * Arguments: G (device arrays, read as kbe_sigma_2b reads them); U device
 * [N][N][N][N] real, U[i][f][d][e] = U_ifde (the index order of Eq. SE; the
 * Hartree-Fock term of Eq. eps pairs its indices as chemists' two-electron
 * integrals (ij|kl)); 0 <= n < G->nt; out device arrays (overwritten); ws a
 * device workspace of kbe_sigma_gf2_workspace(N) bytes (zero-padded copies of
 * U and Uex, rewritten by every call).
 * Errors: KBE_EINVAL (NULL, bad shape), KBE_ERANGE (n), KBE_ENOMEM (ws).
 * ------------------------------------------------------------------------- */
size_t kbe_sigma_gf2_workspace(int32_t N);
kbe_status kbe_sigma_gf2(const kbe_green *G, const double *U, int32_t n, const kbe_sigma_row *out,
                         void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_collision — history integrals at t = t_n for t' = t_m, m in [m0, m1)
 * (the integrals of Eq. KBE2, lesser form, and of Eq. KBE3):
 *   IR[m-m0]  = sum_{s=0}^{n} w[n][s] Sigma^R(t_n,t_s) G^<(t_s,t_m)
 *   IL[m-m0]  = sum_{s=0}^{m} w[m][s] Sigma^<(t_n,t_s) G^R(t_m,t_s)^dagger
 *               (G^A(s,t') = G^R(t',s)^dagger; s = m uses rdiag[m])
 *   Itv[m-m0] = -i sum_j wtau[j] Sigma^](t_n,tau_j) G^](t_m,tau_{J-j})^dagger
 *   Jtv[j]    = sum_{s=0}^{n} w[n][s] Sigma^R(t_n,t_s) G^](t_s,tau_j)
 *             + sum_l Sigma^](t_n,tau_l) C(l,j),   J = ntau-1,
 *     C(l,j) = -wtau_fwd[j][l] G^M(beta+tau_l-tau_j)        for l <= j
 *            + wtau_fwd[J-j][J-l] G^M(tau_l-tau_j)          for l >= j
 *   (the Matsubara convolution of Eq. KBE3 split at tau_j, where G^M jumps;
 *   on [0, tau_j] antiperiodicity gives G^M(x) = -G^M(x+beta)).
 * Selected by flags (KBE_OUT_*); unselected outputs may be NULL and are not
 * written.  KBE_FORCE_GENERIC selects the vector-ALU kernels.
 *
 * Arguments: G; S the self-energy row at t_n; W weights for the same grid;
 * 0 <= n < G->nt; 0 <= m0 <= m1 <= n+1; outputs IR/IL/Itv device
 * [m1-m0][N][N], Jtv device [ntau][N][N] (overwritten); ws device workspace of
 * kbe_collision_workspace(...) bytes.
 * Errors: KBE_EINVAL, KBE_ERANGE, KBE_ENOMEM as above.
 * ------------------------------------------------------------------------- */
size_t kbe_collision_workspace(int32_t N, int32_t nt, int32_t ntau, int32_t n, int32_t m0,
                               int32_t m1, uint32_t flags);
kbe_status kbe_collision(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W, int32_t n,
                         int32_t m0, int32_t m1, uint32_t flags, kbe_c128 *IR, kbe_c128 *IL,
                         kbe_c128 *Itv, kbe_c128 *Jtv, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_collision_both — the lesser and the greater form of Eq. KBE2 from one
 * pass over the history (the call the propagations make at every evaluation:
 * the paper propagates G^< above the diagonal by the lesser form and G^> below
 * it by the greater form, Sec. "Kadanoff Baym Equations").
 *
 * Outputs IR, IL, Itv, Jtv as kbe_collision's lesser form with KBE_OUT_ALL,
 * and IRg, ILg as its greater form's I^R and I^< (KBE_GREATER).  The terms the
 * forms share (I^R's G^< part, I^]) are computed once, the greater form's own
 * terms (the G^R part of G^>, and Sigma^> = Sigma^R + Sigma^< in I^<) are added
 * as further term classes of the same persistent launch, so the upper triangle
 * of kp is read as often as by the lesser form alone.  Each output equals the
 * separate call's to rounding (the partial sums are grouped differently).
 *
 * Arguments: as kbe_collision with flags KBE_OUT_ALL (S needs ret, les and, with
 * ntau > 0, tv; W needs w and, with ntau > 0, wtau and wtau_fwd); IR, IL, IRg,
 * ILg device [m1-m0][N][N]; Itv device [m1-m0][N][N] and Jtv device
 * [ntau][N][N] when ntau > 0 (else ignored); ws device workspace of
 * kbe_collision_both_workspace(...) bytes.  Always the default kernel path.
 * Errors: as kbe_collision.
 * ------------------------------------------------------------------------- */
size_t kbe_collision_both_workspace(int32_t N, int32_t nt, int32_t ntau, int32_t n, int32_t m0,
                                    int32_t m1);
kbe_status kbe_collision_both(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W,
                              int32_t n, int32_t m0, int32_t m1, kbe_c128 *IR, kbe_c128 *IL,
                              kbe_c128 *Itv, kbe_c128 *Jtv, kbe_c128 *IRg, kbe_c128 *ILg,
                              void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_collision_both_vjp — adjoint of kbe_collision_both (the propagations'
 * adjoint call).
 *
 * By linearity the gradient is the lesser form's adjoint with the summed
 * cotangents of the terms the forms share (gIR + gIRg, gIL + gILg, gItv, gJtv)
 * plus the adjoint of the greater form's own terms (the G^R part of G^> in I^R,
 * the Sigma^R part of Sigma^> in I^<) with gIRg and gILg: two passes over the
 * history for the self-energy gradients, and for the Green's-function gradient
 * one pass that writes each block once with both sets of terms (N = 16 and
 * 5 <= N <= 8; two at other N).
 *
 * Arguments: as kbe_collision_both for G, S, W, n, m0, m1; the cotangents gIR,
 * gIL, gIRg, gILg [m1-m0][N][N], gItv [m1-m0][N][N] and gJtv [ntau][N][N]
 * (both when ntau > 0); gG (G's shape) receives the Green's-function gradient
 * by accumulation (there is no overwrite mode: the greater form's terms reach
 * blocks outside the lesser form's); gS (ret, les [n+1][N][N], tv [ntau][N][N])
 * is overwritten with the self-energy gradient; ws: device workspace of
 * kbe_collision_both_vjp_workspace(...) bytes.  Complex gradients as in
 * kbe_collision_vjp.  Errors: as kbe_collision_vjp.
 * ------------------------------------------------------------------------- */
size_t kbe_collision_both_vjp_workspace(int32_t N, int32_t nt, int32_t ntau, int32_t n,
                                        int32_t m0, int32_t m1);
kbe_status kbe_collision_both_vjp(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W,
                                  int32_t n, int32_t m0, int32_t m1, const kbe_c128 *gIR,
                                  const kbe_c128 *gIL, const kbe_c128 *gItv,
                                  const kbe_c128 *gJtv, const kbe_c128 *gIRg,
                                  const kbe_c128 *gILg, const kbe_green *gG,
                                  const kbe_sigma_row *gS, void *ws, size_t ws_bytes,
                                  void *stream);

/* ---------------------------------------------------------------------------
 * kbe_collision_noalloc — kbe_collision for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same integrals, arguments and errors as
 * kbe_collision, without the workspace arguments.  The workspace lives in a
 * fixed device array of KBE_NOALLOC_SCRATCH_BYTES inside the library; every
 * device the library runs on holds its own copy until the process ends.  The
 * call allocates nothing: it enqueues the same kernels as kbe_collision on
 * `stream`, using that device's array.
 *
 * All calls on one device share its array and every call overwrites it (what
 * must start at zero is cleared by the call itself, on the stream), so calls
 * that may overlap on one device race: issue them on one stream, or order them.
 * The first call on a device looks up the array's device address (a host-side
 * query, no allocation).
 * Errors: as kbe_collision, plus KBE_ENOMEM when the call would need more than
 * KBE_NOALLOC_SCRATCH_BYTES of workspace (kbe_collision_workspace() tells; the
 * 8-orbital history of 1024 points with 256 tau points needs 29 MiB, the
 * 16-orbital one of 2048 points needs 232 MiB and is rejected).
 * ------------------------------------------------------------------------- */
#define KBE_NOALLOC_SCRATCH_BYTES (64u << 20) /* 64 MiB per device */
kbe_status kbe_collision_noalloc(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W,
                                 int32_t n, int32_t m0, int32_t m1, uint32_t flags, kbe_c128 *IR,
                                 kbe_c128 *IL, kbe_c128 *Itv, kbe_c128 *Jtv, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_collision_vjp — adjoint of kbe_collision (a project addition to the
 * paper's method, used for gradients of observables).
 *
 * Complex gradients follow PyTorch's convention: for a real loss L and a
 * complex variable z the gradient is dL/dRe z + i dL/dIm z.  Given the
 * cotangents gIR, gIL, gItv ([m1-m0][N][N]) and gJtv ([ntau][N][N]) of the
 * outputs selected by flags, the call
 *   - overwrites gS (the gradient of the self-energy row: ret and les
 *     [n+1][N][N], tv [ntau][N][N]), and
 *   - adds the gradient of the Green's function into gG (kp, rdiag, tv, mat),
 *     or overwrites the blocks the forward call reads when flags contains
 *     KBE_GRAD_OVERWRITE (blocks it does not read are left untouched).
 * Weights are not differentiated (they depend only on the grid).
 *
 * Arguments: as kbe_collision; gG must have G's shape; cotangents of
 * unselected outputs may be NULL.  ws: kbe_collision_vjp_workspace(...) bytes.
 * Errors: as kbe_collision.
 * ------------------------------------------------------------------------- */
size_t kbe_collision_vjp_workspace(int32_t N, int32_t nt, int32_t ntau, int32_t n, int32_t m0,
                                   int32_t m1, uint32_t flags);
kbe_status kbe_collision_vjp(const kbe_green *G, const kbe_sigma_row *S, const kbe_wts *W,
                             int32_t n, int32_t m0, int32_t m1, uint32_t flags,
                             const kbe_c128 *gIR, const kbe_c128 *gIL, const kbe_c128 *gItv,
                             const kbe_c128 *gJtv, const kbe_green *gG, const kbe_sigma_row *gS,
                             void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_sigma_2b_vjp — adjoint of kbe_sigma_2b (project addition).
 *
 * Given gS (the cotangent of the row: ret/les [n+1][N][N], tv [ntau][N][N]),
 * adds the gradient with respect to G into gG (row n and column n of kp,
 * rdiag[n], tv[n]) and the gradient with respect to the real interaction u
 * into gu (device [N]).  The self-energy is recomputed from G, not stored.
 * ws: kbe_sigma_2b_vjp_workspace(...) bytes (a deterministic reduction of gu).
 * Errors: as kbe_sigma_2b, plus KBE_ENOMEM.
 * ------------------------------------------------------------------------- */
size_t kbe_sigma_2b_vjp_workspace(int32_t N, int32_t n, int32_t ntau);
kbe_status kbe_sigma_2b_vjp(const kbe_green *G, const double *u, int32_t n,
                            const kbe_sigma_row *gS, const kbe_green *gG, double *gu, void *ws,
                            size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Batches of history rows (a project addition: many independent rows of
 * different systems, orbital counts and lengths in one launch).
 *
 * An item is one row (t_n, t_m) of one system, given by the blocks that row
 * reads (its "cross" storage), all device memory with the item's own N:
 *   sig_ret, sig_les [n+1]  Sigma^R(t_n,t_s), Sigma^<(t_n,t_s), s = 0..n
 *   sig_tv  [ntau]          Sigma^](t_n,tau_j)
 *   col     [m+1]           kp[s][m] = G^<(t_s,t_m), s = 0..m (block s at
 *                           col + s * max(col_ld, 1) blocks)
 *   row     [n+1]           kp[m][s]: G^R(t_m,t_s) for s < m, G^<(t_m,t_s) for s >= m
 *   rdiag   [1]             G^R(t_m,t_m)
 *   tv      [ntau]          G^](t_m,tau_j)
 *   wn [n+1], wm [m+1]      weight rows w[n][.] and w[m][.]; wtau [ntau]
 * and it asks for the integrals of kbe_collision at that single (n, m):
 *   IR  = sum_{s<=m} wn[s] sig_ret[s] col[s] - sum_{s>m} wn[s] sig_ret[s] row[s]^dagger
 *   IL  = sum_{s<m} wm[s] sig_les[s] row[s]^dagger + wm[m] sig_les[m] rdiag^dagger
 *   Itv = -i sum_j wtau[j] sig_tv[j] tv[J-j]^dagger
 * (G^<(t_s,t_m) = -kp[m][s]^dagger for s > m; these are a3-a5 of kbe_collision
 * with the row's blocks passed directly).  Outputs are one N x N block each.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t N;     /* orbitals, 1..KBE_NMAX */
  int32_t n, m;  /* row and column, 0 <= m <= n */
  int32_t ntau;  /* imaginary-time points: 0 or >= 2 */
  uint32_t flags; /* KBE_OUT_IR | KBE_OUT_IL | KBE_OUT_ITV (J^] is not a per-row output) */
  int32_t chunk;  /* terms per work unit for this item: 0 (the library default, 64) or 32, 64,
                     128, 256; used when the call's chunk is 0 (kbe_collision_batch_tune_groups
                     writes it) */
  const kbe_c128 *sig_ret, *sig_les, *sig_tv;
  const kbe_c128 *col, *row, *rdiag, *tv;
  const double *wn, *wm, *wtau;
  kbe_c128 *IR, *IL, *Itv; /* one block each; NULL when its flag is off */
  int64_t col_ld;          /* blocks from col[s] to col[s+1]: 0 or 1 for a contiguous array;
                              the system's ldt to read column m of its KP storage in place
                              (col = kp + m blocks) */
} kbe_batch_item;

#define KBE_BATCH_MAX 65536 /* most items per call */

/* ---------------------------------------------------------------------------
 * kbe_collision_batch — the items' integrals in one persistent launch.
 *
 * items: host array of count items (validated here); items_dev: the same array
 * copied by the caller into device memory (what the kernels read; its content
 * must equal items when the work runs).  chunk: terms per work unit for every
 * item, one of 32, 64, 128, 256; or 0, when each item's own chunk field applies
 * (see kbe_collision_batch_tune and kbe_collision_batch_tune_groups).
 * ws: kbe_collision_batch_workspace(items, count, chunk) bytes.  Nothing is
 * copied from host memory and nothing is allocated, so the call can be
 * captured in a HIP graph and replayed.
 * Errors: KBE_EINVAL (NULL pointers, N out of range, bad flags, chunk not
 * allowed), KBE_ERANGE (m > n, negative sizes, count > KBE_BATCH_MAX),
 * KBE_ENOMEM (workspace too small).
 * ------------------------------------------------------------------------- */
size_t kbe_collision_batch_workspace(const kbe_batch_item *items, int32_t count, int32_t chunk);
kbe_status kbe_collision_batch(const kbe_batch_item *items, const kbe_batch_item *items_dev,
                               int32_t count, int32_t chunk, void *ws, size_t ws_bytes,
                               void *stream);

/* ---------------------------------------------------------------------------
 * kbe_collision_batch_tune — the autotuner: runs kbe_collision_batch on the
 * given batch once per allowed chunk size (after one warm-up call each), times
 * each with HIP events on the stream, and returns the fastest in *best_chunk
 * (and, if times_ms is not NULL, the four times in the order 32, 64, 128,
 * 256).  It synchronises the stream.  ws must hold the workspace of the
 * largest requirement (chunk = 32).  Errors: as kbe_collision_batch, plus
 * KBE_EHIP.
 * ------------------------------------------------------------------------- */
kbe_status kbe_collision_batch_tune(const kbe_batch_item *items, const kbe_batch_item *items_dev,
                                    int32_t count, void *ws, size_t ws_bytes, void *stream,
                                    int32_t *best_chunk, float *times_ms);

/* ---------------------------------------------------------------------------
 * kbe_collision_batch_tune_groups — the autotuner's tile table: a chunk size
 * per group of items, a group being the items of one N and one length bucket
 * floor(log2(n + 1)).  It starts from the best common chunk and makes two
 * coordinate-descent passes, first over the groups of one N, then over the
 * groups of one N and one length bucket: for each group in decreasing order of
 * its bytes it tries the other chunk sizes on that group's items alone and keeps
 * one only if the whole call (best of three timed calls after a warm-up) gets
 * faster by more than 1%.  On return every item's
 * chunk field holds its group's chunk, in items and (copied by this call) in
 * items_dev, so kbe_collision_batch(..., chunk = 0, ...) runs the table; the
 * caller may read the fields back to store the table.  *best_ms (if not NULL)
 * receives the tuned call's time.  It synchronises the stream.  ws: as for
 * kbe_collision_batch_tune.  Errors: as kbe_collision_batch_tune.
 * ------------------------------------------------------------------------- */
kbe_status kbe_collision_batch_tune_groups(kbe_batch_item *items, kbe_batch_item *items_dev,
                                           int32_t count, void *ws, size_t ws_bytes, void *stream,
                                           float *best_ms);

/* ---------------------------------------------------------------------------
 * kbe_collision_batch_vjp — the adjoint of kbe_collision_batch (a project
 * addition, for gradients through batches of rows).
 *
 * An item is a row as for kbe_collision_batch (its IR, IL, Itv are not used),
 * the cotangents of the row's selected outputs, and the gradient arrays of the
 * row's inputs.  Complex gradients follow PyTorch's convention (dL/dRe + i
 * dL/dIm).  Each input block of a row enters exactly one term of one output,
 * c A B or c A B^dagger, which gives it the gradient conj(c) g B^dagger,
 * conj(c) A^dagger g (for c A B) or conj(c) g B, c g^dagger A (for
 * c A B^dagger); so, with GR, GL, GT the cotangents of IR, IL, Itv:
 *   g_sig_ret[s] = wn[s] GR col[s]^dagger (s <= m),  -wn[s] GR row[s] (s > m)
 *   g_col[s]     = wn[s] sig_ret[s]^dagger GR                    (s <= m)
 *   g_row[s]     = -wn[s] GR^dagger sig_ret[s] (s > m),  wm[s] GL^dagger sig_les[s] (s < m)
 *   g_sig_les[s] = wm[s] GL row[s] (s < m),  wm[m] GL rdiag (s = m)
 *   g_rdiag      = wm[m] GL^dagger sig_les[m]
 *   g_sig_tv[j]  = i wtau[j] GT tv[J-j],  g_tv[J-j] = -i wtau[j] GT^dagger sig_tv[j]
 * Every gradient block is overwritten; blocks no selected output reads
 * (g_sig_les[s > m], g_row[m], and those of unselected outputs) are set to 0.
 * No reduction is involved, so results do not depend on the schedule.
 *
 * items: host array (validated here); items_dev: the same array in device
 * memory, read by the kernels; ws: kbe_collision_batch_vjp_workspace(count)
 * bytes.  Nothing is copied from host memory and nothing is allocated, so the
 * call can be captured in a HIP graph.
 * Errors: KBE_EINVAL (NULL pointers, N out of range, bad flags), KBE_ERANGE
 * (m > n, negative sizes, count > KBE_BATCH_MAX), KBE_ENOMEM (workspace).
 * ------------------------------------------------------------------------- */
typedef struct {
  kbe_batch_item row;               /* the row, as for kbe_collision_batch */
  const kbe_c128 *gIR, *gIL, *gItv; /* cotangents, one N x N block each (NULL when the flag is off) */
  kbe_c128 *g_sig_ret, *g_sig_les;  /* [n+1] each */
  kbe_c128 *g_sig_tv;               /* [ntau] (may be NULL when ntau == 0) */
  kbe_c128 *g_col;                  /* [m+1] */
  kbe_c128 *g_row;                  /* [n+1] */
  kbe_c128 *g_rdiag;                /* [1] */
  kbe_c128 *g_tv;                   /* [ntau] (may be NULL when ntau == 0) */
} kbe_batch_vjp_item;

size_t kbe_collision_batch_vjp_workspace(int32_t count);
kbe_status kbe_collision_batch_vjp(const kbe_batch_vjp_item *items,
                                   const kbe_batch_vjp_item *items_dev, int32_t count, void *ws,
                                   size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Fixed-grid propagation of the Kadanoff-Baym equations and its adjoint (a
 * project addition built on the hot path: gradients of observables with
 * respect to the interaction and a drive, through a whole propagation).
 *
 * The paper propagates G^< above the diagonal (Eq. KBE1), G^> below it
 * (Eq. KBE2) and G^] (Eq. KBE3) as one growing state vector (Sec. "Adaptive
 * Time Stepping"); here the grid and the orders are fixed.  The unknowns are
 * the KP storage of G: at step n the new column kp[m][n] = G^<(t_m,t_n)
 * (m <= n), the new row kp[n][m] = G^R(t_n,t_m) (m < n) and tv[n][j]; each
 * block obeys an ODE in t_n whose right side takes the history sums of
 * kbe_collision in the lesser form (C^< = I^R + I^< + I^]) and the greater
 * form (C^>), J^] of Eq. KBE3, the second-Born row of kbe_sigma_2b and the
 * Fock matrix of Eq. eps for a local interaction with a Gaussian pulse:
 *   eps(t) = h0 + A exp(-(t - t0)^2 / (2 s^2)) e_00 + diag(-i u_i G^<_ii(t,t)),
 *   d/dt_n kp[m][n] = i (kp[m][n] eps - C^<(n,m)^dagger)                (m < n)
 *   d/dt_n kp[n][m] = -i (eps kp[n][m] + C^>(n,m) - C^<(n,m))           (m < n)
 *   d/dt_n kp[n][n] = -i [eps, kp[n][n]] - i (C^<(n,n) + C^<(n,n)^dagger)
 *   d/dt_n tv[n][j] = -i (eps tv[n][j] + J^](n,j)).
 * kp[m][.] and kp[.][m] start at t_m from kp[m][m] and -i.  Every block
 * advances over [t_{n-1}, t_n] by the implicit Adams-Moulton rule in Lagrange
 * form with the local weights of Eq. weights on min(order[n], n - b + 1)
 * nodes (b: the step where the block's history begins), solved by `iters`
 * fixed-point iterations from an explicit Euler predictor; the right sides
 * kept for later steps are evaluated once more at the accepted values.  The
 * initial state follows Eq. BC: rdiag = -i 1, and with a thermal branch
 * tv[0][j] = -i G^M(beta - tau_j) = -i mat[ntau-1-j] and
 * kp[0][0] = -tv[0][0]^dagger; without one, kp[0][0] = G^<(0,0) = i rho(0)
 * is read from G.  The observable is the density n_i(t_n) = Re(-i G^<_ii).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t iters;         /* fixed-point iterations per step, >= 1 */
  const double *h0;      /* device [N][N], real symmetric */
  const double *u;       /* device [N], local interaction (a scalar U fills every entry) */
  double pulse_amp;      /* A */
  double pulse_t0;       /* centre t0 */
  double pulse_sigma;    /* width s > 0 */
  const double *t;       /* device [nt], the grid (t[0] = 0) */
  const int32_t *order;  /* device [nt], nodes per interval (as in kbe_grid) */
  const double *lam;     /* device [nt][KBE_KMAX][KBE_KMAX], from kbe_step_weights(t, order) */
} kbe_prop;

/* kbe_propagate: runs the propagation over the whole grid.  G (device, N,
 * nt, ntau, ldt as for the other calls): mat holds G^M (read); kp, rdiag, tv
 * are written with the solution (kp[0][0] read first when ntau == 0).  W: the
 * weights of the same grid (kbe_weights / kbe_weights_dev).  dens: device
 * [nt][N] output, n_i(t_n).  ws: kbe_propagate_workspace(...) bytes; it keeps
 * the right-side history and the fixed-point iterates that
 * kbe_propagate_vjp needs.  Errors: KBE_EINVAL (NULL pointers, bad shapes,
 * iters < 1, pulse_sigma <= 0), KBE_ENOMEM (workspace). */
size_t kbe_propagate_workspace(int32_t N, int32_t nt, int32_t ntau, int64_t ldt, int32_t iters);
kbe_status kbe_propagate(const kbe_prop *P, const kbe_wts *W, const kbe_green *G, double *dens,
                         void *ws, size_t ws_bytes, void *stream);

/* kbe_propagate_vjp: the adjoint of kbe_propagate.  Given gdens (device
 * [nt][N], the gradient of a real loss with respect to dens), writes
 * gu (device [N]) = dL/du_i and gamp (device, one double) = dL/dA, exact
 * derivatives of the discrete propagation (every self-energy row is
 * recomputed from the stored iterates; the collision and self-energy adjoints
 * run on the same kernels as kbe_collision_vjp and kbe_sigma_2b_vjp).  P, W,
 * G and ws must be those of the kbe_propagate call, unchanged since: G holds
 * the solution again when the call returns.  Errors: as kbe_propagate. */
kbe_status kbe_propagate_vjp(const kbe_prop *P, const kbe_wts *W, const kbe_green *G,
                             const double *gdens, double *gu, double *gamp, void *ws,
                             size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_propagate_adaptive — the adaptive propagation (Sec. "Adaptive Time
 * Stepping" and Sec. "Adaptive History Integration"): the stacked state of
 * kbe_propagate advanced by variable-step, variable-order Adams methods on a
 * grid that grows by one point per accepted step.
 *
 * Step n (from t_{n-1} by h, order q <= min(qmax, n)) for every block: the
 * predictor integrates over [t_{n-1}, t_n] the interpolant of the block's right
 * sides at t_{n-q..n-1}; the corrector is the Adams-Moulton rule of order q
 * (the local weights of Eq. weights on t_{n-q+1..n}), solved by fixed-point
 * iteration (at most maxcor corrections; converged when
 * min(1, R_m) d_m C < 0.1 with d_m the WRMS norm of the last correction,
 * R_m = max(0.3 R_{m-1}, d_m / d_{m-1}), R_1 = 1, and C the error-estimate
 * coefficient; a diverging or non-converged iteration retries with h / 4).
 * Before every evaluation of the right sides the history order is chosen: the
 * test integral of G^R(t_n,s) Sigma^<(s,t_n) + G^<(t_n,s) Sigma^A(s,t_n) over
 * [t_{n-1}, t_n] with k = 1..min(kmax, n+1) nodes, k_opt the first minimiser
 * of ||I^(k) - I^(k-1)||_F over k >= 2, and row n of the history weights is
 * row n-1 plus the local weights on k_opt nodes.  The local error is
 * C (y_n - y_pred) with C = |c_AM / (c_AB - c_AM)| from the principal error
 * coefficients of the corrector and the predictor (Milne's device), measured
 * in the WRMS norm of Eq. wrms_norm with the weights of Eq. ewt
 * (1 / (rtol |y_{n-1}| + atol), per complex entry); E > 1 rejects the step
 * (h times max(0.2, min(0.9, 0.9 E^(-1/(q+1)))); q = 1 and h / 4 after three
 * rejections).  After an accepted step the right sides are evaluated at the
 * accepted values, and those of the blocks born at t_n (kp[.][n], kp[n][.])
 * are reconstructed at the qmax points below the diagonal from the history
 * sums of Eq. KBE2 at rows j < n (Sec. "Implementation": the equations hold on
 * both sides of the diagonal), so every block has a history of q points.  The
 * next step: eta_q = 1 / ((6 E)^(1/(q+1)) + 1e-6) and, once q+1 steps were
 * taken at order q, eta_{q-1}, eta_{q+1} from the WRMS norms of the
 * corresponding error coefficients times divided differences of the right
 * sides (biases 6 and 10); the largest wins (q on ties); below 1.5 nothing
 * changes, else h grows by at most 10.  The last step ends at t_end.
 *
 * Arguments: P as for kbe_propagate (t, order and lam are not used: the grid
 * is built here); C the controls; W: wtau and wtau_fwd of the tau grid (W->w
 * is not used: the history weights are built in the workspace); G with
 * capacity G->nt points (mat read; kp, rdiag, tv written; kp[0][0] read when
 * ntau == 0); dens device [G->nt][N] (rows 0..trace->nt-1 written); trace:
 * host arrays of G->nt entries (ks: G->nt x (12 + 2)), filled by the call;
 * ws: kbe_propagate_adaptive_workspace(N, G->nt, ntau) bytes.  The call
 * synchronises the stream at every fixed-point iteration (the controller
 * reads the norms).  Errors: KBE_EINVAL (NULL pointers, bad controls),
 * KBE_ENOMEM (workspace), KBE_EHIP, KBE_ESTEP (the step size fell below
 * 1e-13 max(1, t), or G->nt points were accepted before t_end: trace, dens
 * and G hold the accepted steps, trace->nt of them).
 * ------------------------------------------------------------------------- */
typedef struct {
  double t_end;    /* final time > 0 */
  double rtol;     /* relative tolerance > 0 */
  double atol;     /* absolute tolerance > 0 */
  double h0;       /* first step > 0 */
  int32_t qmax;    /* largest Adams order, 1..12 */
  int32_t kmax;    /* largest history order K, 2..KBE_KMAX */
  int32_t maxcor;  /* fixed-point corrections per attempt, 1..12 */
} kbe_adapt_ctl;

typedef struct {
  double *t;         /* [capacity] accepted grid */
  int32_t *q;        /* [capacity] Adams order of step n (q[0] = 0) */
  int32_t *m;        /* [capacity] fixed-point iterations of step n */
  int32_t *ks;       /* [capacity][14] history order of each evaluation of step n (m + 1) */
  double *err;       /* [capacity] error norm E of step n */
  int32_t nt;        /* out: points of the grid (steps + 1) */
  int32_t rejected;  /* out: rejected attempts */
} kbe_adapt_trace;

size_t kbe_propagate_adaptive_workspace(int32_t N, int32_t capacity, int32_t ntau);
kbe_status kbe_propagate_adaptive(const kbe_prop *P, const kbe_adapt_ctl *C, const kbe_wts *W,
                                  const kbe_green *G, double *dens, kbe_adapt_trace *trace,
                                  void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * kbe_equilibrium — an interacting equilibrium initial state G^M: the
 * Matsubara Dyson equation of the local-U second-Born approximation (a project
 * addition: the paper takes G^M as given, Sec. "Kadanoff Baym Equations").
 *
 * In equilibrium Eq. KBE3 at t = 0, with the boundary conditions of Eq. BC
 * (G^](0,tau) = i G^M(-tau), Sigma^](0,tau) = i Sigma^M(-tau)), becomes
 * -dG^M/dtau = eps G^M + int_0^beta Sigma^M(u) G^M(tau - u) du, antiperiodic in
 * tau; its integral form G^M = G0 + G0 * Sigma^M * G^M is solved by mixed
 * fixed-point iteration from the free function of h0 - mu:
 *   eps = h0 + diag(u_i n_i) - mu with n_i = -G^M_ii(beta-) (the Hartree term
 *   of Eq. eps), G0(tau) = -exp(-eps tau)(1 - f(eps)) (eigendecomposition of
 *   eps), Sigma^M_ij(tau) = u_i u_j G^M_ij(tau)^2 G^M_ji(beta - tau) (Eq. SE at
 *   t = 0), Gn = G0 + G0 * (Sigma^M * G^M), G^M <- (1 - mix) G^M + mix Gn,
 * until the largest |Gn - G^M| is below tol.  Each * is the integral over
 * [0, beta] split at u = tau_j: wtau_fwd[j][l] A(tau_{j-l}) B(tau_l) summed over
 * l <= j, minus wtau_fwd[J-j][J-l] A(tau_{J+j-l}) B(tau_l) summed over l >= j
 * (the rule over [tau_j, beta] by reflection, the part above tau_j continued
 * antiperiodically).  A propagation started from the result is stationary up to
 * its time-stepping error, which the free G^M of an interacting system is not.
 *
 * Arguments: N orbitals (1..KBE_NMAX); ntau >= 2 points tau_j = j beta /
 * (ntau - 1) (tau_0 = 0+, tau_J = beta-), beta > 0; wtau_fwd device
 * [ntau][ntau] from kbe_weights / kbe_weights_dev for this tau grid; h0 device
 * [N][N] real symmetric (its symmetric part is used); u device [N]; C: mu, mix
 * in (0, 1], tol > 0, maxit >= 1 (in), iterations and change (out: the
 * iterations run and the last largest change); mat device [ntau][N][N]
 * (written: G^M, real); ws: kbe_equilibrium_workspace(N, ntau) bytes.  The
 * call synchronises the stream once per iteration (to read the change).
 * Errors: KBE_EINVAL (NULL pointers, N, ntau, beta or controls out of range),
 * KBE_ENOMEM (workspace), KBE_EHIP, KBE_ECONV (change still >= tol after maxit
 * iterations, or not finite: mat holds the last iterate).
 * ------------------------------------------------------------------------- */
typedef struct {
  double mu;          /* chemical potential */
  double mix;         /* weight of the new iterate, 0 < mix <= 1 */
  double tol;         /* convergence: largest change of an element below tol, > 0 */
  int32_t maxit;      /* iteration limit, >= 1 */
  int32_t iterations; /* out: iterations run */
  double change;      /* out: largest |Gn - G^M| of the last iteration */
} kbe_eq_ctl;

size_t kbe_equilibrium_workspace(int32_t N, int32_t ntau);
kbe_status kbe_equilibrium(int32_t N, int32_t ntau, double beta, const double *wtau_fwd,
                           const double *h0, const double *u, kbe_eq_ctl *C, kbe_c128 *mat,
                           void *ws, size_t ws_bytes, void *stream);

/* Human-readable name of a status code (static string). */
const char *kbe_status_string(kbe_status s);
/* Detail of the last error on the calling thread ("" if none). */
const char *kbe_last_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int32_t kbe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KBE_H */
