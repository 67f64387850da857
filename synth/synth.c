/*
 * Seeded synthetic inputs for the history-integral path.
 *
 * This file draws random numbers and lays them out; it holds none of the
 * method's arithmetic (no weights, no self-energy, no integrals).  Both the
 * GPU library's tests/benchmark and the CPU oracle's tests consume its output,
 * so the two sides always see bit-identical inputs.
 *
 * Generator: counter-based.  Every value is a pure function of
 * (seed, stream id, logical element index), so any sub-range of an array can
 * be produced independently and in parallel, and the content does not depend
 * on the leading dimension the caller stores it with.
 *   - mixing function: the SplitMix64 output finaliser (Steele, Lea & Flood,
 *     "Fast splittable pseudorandom number generators", OOPSLA 2014),
 *   - uniform: top 53 bits of the mixed word, scaled to [0, 1),
 *   - normal pair: the Box-Muller transform (Box & Muller 1958).
 *
 * Complex entries are stored as interleaved (re, im) doubles (complex128).
 * Blocks are N x N, row-major.  Two-time arrays use the "KP" layout:
 *   kp[a][b] (a <= b) holds G^<(t_a, t_b); kp[a][b] (a > b) holds G^R(t_a, t_b);
 * see include/kbe.h for the full statement of the layout.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed + GOLDEN) ^ (stream * 0xd1b54a32d192ed03ULL + 0x632be59bd9b4e019ULL));
}

static inline double uniform01(uint64_t key, uint64_t idx) {
  return (double)(mix64(key + (idx + 1) * GOLDEN) >> 11) * 0x1.0p-53;
}

/* One complex value with independent N(0,1) real and imaginary parts. */
static inline void normal_pair(uint64_t key, uint64_t idx, double *re, double *im) {
  double u1 = uniform01(key, 2 * idx);
  double u2 = uniform01(key, 2 * idx + 1);
  double r = sqrt(-2.0 * log(1.0 - u1));
  double th = 6.283185307179586476925286766559 * u2;
  *re = r * cos(th);
  *im = r * sin(th);
}

/* Stream ids: one per array so that arrays are uncorrelated. */
enum { S_STEP = 1, S_ORDER = 2, S_KP = 3, S_TV = 4, S_MAT = 5, S_SIG_R = 6, S_SIG_L = 7,
       S_SIG_TV = 8, S_COT = 9 };

/* Grid: t[0] = 0, t[p] = t[p-1] + h_p with h_p ~ U[hmin, hmax];
 * order[p] ~ U{omin..omax} for p >= 1, order[0] = omin (unused). */
void synth_grid(uint64_t seed, int32_t nt, double hmin, double hmax, int32_t omin, int32_t omax,
                double *t, int32_t *order) {
  uint64_t ks = stream_key(seed, S_STEP), ko = stream_key(seed, S_ORDER);
  t[0] = 0.0;
  order[0] = omin;
  for (int32_t p = 1; p < nt; ++p) {
    t[p] = t[p - 1] + hmin + (hmax - hmin) * uniform01(ks, (uint64_t)p);
    int32_t span = omax - omin + 1;
    int32_t o = omin + (int32_t)(uniform01(ko, (uint64_t)p) * span);
    if (o > omax) o = omax;
    order[p] = o;
  }
}

/* Make an N x N block anti-Hermitian: X <- (X - X^H)/2. */
static void anti_hermitian(double *blk, int32_t N) {
  for (int32_t i = 0; i < N; ++i)
    for (int32_t j = i; j < N; ++j) {
      double *x = blk + 2 * (i * N + j), *y = blk + 2 * (j * N + i);
      double re = 0.5 * (x[0] - y[0]), im = 0.5 * (x[1] + y[1]);
      x[0] = re; x[1] = im;          /* x = (x - conj(y))/2 */
      y[0] = -re; y[1] = im;         /* y = -conj(x) */
    }
}

static void fill_block(uint64_t key, uint64_t base, int32_t N, double scale, double *blk) {
  for (int32_t e = 0; e < N * N; ++e) {
    double re, im;
    normal_pair(key, base + (uint64_t)e, &re, &im);
    blk[2 * e] = scale * re;
    blk[2 * e + 1] = scale * im;
  }
}

/* Two-time array in KP layout for rows a in [a0, a1), all columns b < nt.
 * Every block is N(0,1) times exp(-decay |t_a - t_b|); diagonal blocks are
 * made anti-Hermitian (the lesser symmetry at equal times).  out points at
 * row a0 (out + ((a - a0) * ldt + b) * N * N * 2 doubles). */
void synth_kp_rows(uint64_t seed, int32_t N, int32_t nt, int64_t ldt, const double *t, double decay,
                   int32_t a0, int32_t a1, double *out) {
  uint64_t key = stream_key(seed, S_KP);
  int64_t bs = (int64_t)N * N;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t a = a0; a < a1; ++a) {
    for (int32_t b = 0; b < nt; ++b) {
      double *blk = out + 2 * (((int64_t)(a - a0) * ldt + b) * bs);
      double sc = exp(-decay * fabs(t[a] - t[b]));
      fill_block(key, ((uint64_t)a * (uint64_t)nt + (uint64_t)b) * (uint64_t)bs, N, sc, blk);
      if (a == b) anti_hermitian(blk, N);
    }
  }
}

/* One column b of the same KP array, rows a in [a0, a1): block (a, b) exactly as
 * synth_kp_rows makes it (out + (a - a0) * N * N * 2 doubles). */
void synth_kp_col(uint64_t seed, int32_t N, int32_t nt, const double *t, double decay, int32_t b,
                  int32_t a0, int32_t a1, double *out) {
  uint64_t key = stream_key(seed, S_KP);
  int64_t bs = (int64_t)N * N;
#pragma omp parallel for schedule(static)
  for (int32_t a = a0; a < a1; ++a) {
    double *blk = out + 2 * ((int64_t)(a - a0) * bs);
    double sc = exp(-decay * fabs(t[a] - t[b]));
    fill_block(key, ((uint64_t)a * (uint64_t)nt + (uint64_t)b) * (uint64_t)bs, N, sc, blk);
    if (a == b) anti_hermitian(blk, N);
  }
}

/* Equal-time retarded values G^R(t,t) = -i * identity for rows [0, nt). */
void synth_rdiag(int32_t N, int32_t nt, double *out) {
  int64_t bs = (int64_t)N * N;
  memset(out, 0, sizeof(double) * 2 * (size_t)(nt * bs));
  for (int32_t a = 0; a < nt; ++a)
    for (int32_t i = 0; i < N; ++i) out[2 * (a * bs + i * N + i) + 1] = -1.0;
}

/* Mixed component tv[m][j] for rows m in [m0, m1): N(0,1) times exp(-decay t_m). */
void synth_tv_rows(uint64_t seed, int32_t N, int32_t ntau, const double *t, double decay,
                   int32_t m0, int32_t m1, double *out) {
  uint64_t key = stream_key(seed, S_TV);
  int64_t bs = (int64_t)N * N;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t m = m0; m < m1; ++m) {
    double sc = exp(-decay * t[m]);
    for (int32_t j = 0; j < ntau; ++j)
      fill_block(key, ((uint64_t)m * (uint64_t)ntau + (uint64_t)j) * (uint64_t)bs, N, sc,
                 out + 2 * (((int64_t)(m - m0) * ntau + j) * bs));
  }
}

/* Matsubara component mat[j], N(0,1) entries, no envelope. */
void synth_mat(uint64_t seed, int32_t N, int32_t ntau, double *out) {
  uint64_t key = stream_key(seed, S_MAT);
  int64_t bs = (int64_t)N * N;
  for (int32_t j = 0; j < ntau; ++j)
    fill_block(key, (uint64_t)j * (uint64_t)bs, N, 1.0, out + 2 * (j * bs));
}

/* Self-energy row at t_n given directly (no self-consistency):
 * ret[s], les[s] for s in [0, n] with envelope exp(-decay |t_n - t_s|),
 * les[n] anti-Hermitian; tv[j] for j < ntau with envelope exp(-decay t_n). */
void synth_sigma_row(uint64_t seed, int32_t N, int32_t n, int32_t ntau, const double *t,
                     double decay, double *ret, double *les, double *tv) {
  uint64_t kr = stream_key(seed, S_SIG_R), kl = stream_key(seed, S_SIG_L),
           kt = stream_key(seed, S_SIG_TV);
  int64_t bs = (int64_t)N * N;
  for (int32_t s = 0; s <= n; ++s) {
    double sc = exp(-decay * fabs(t[n] - t[s]));
    fill_block(kr, (uint64_t)s * (uint64_t)bs, N, sc, ret + 2 * (s * bs));
    fill_block(kl, (uint64_t)s * (uint64_t)bs, N, sc, les + 2 * (s * bs));
  }
  anti_hermitian(les + 2 * (n * bs), N);
  double sc = exp(-decay * t[n]);
  for (int32_t j = 0; j < ntau; ++j)
    fill_block(kt, (uint64_t)j * (uint64_t)bs, N, sc, tv + 2 * (j * bs));
}

/* Generic complex N(0,1) array of count elements (cotangents, perturbations);
 * stream lets callers draw several independent arrays from one seed. */
void synth_normal(uint64_t seed, uint64_t stream, int64_t count, double *out) {
  uint64_t key = stream_key(seed, S_COT + 16 * stream);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < count; ++e) normal_pair(key, (uint64_t)e, out + 2 * e, out + 2 * e + 1);
}
