/*
 * Seeded synthetic inputs for the Wilson-Dirac path: gauge links, sources,
 * random SU(3) gauge transformations and uniform test vectors.
 *
 * This file holds no arithmetic of the method itself (no hopping term, no
 * projector, no solver step).  It only draws random numbers and turns them
 * into SU(3) matrices and spinor components.  Both the FP64 oracle and the
 * GPU path are fed from the arrays written here.
 *
 * Random numbers: Philox4x64-10, the counter-based generator of Salmon,
 * Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11).  Every draw is addressed by (seed, stream, index, block), so the
 * output does not depend on the number of threads or on the traversal order.
 * Gaussian pairs use the Box-Muller transform.
 *
 * Link recipe: A is a 3x3 complex Gaussian matrix (re, im ~ N(0,1)),
 * H = (A + A^dagger)/2 with its trace removed, U = exp(i eps H) by a scaled
 * Taylor series with repeated squaring, followed by reunitarization
 * (Gram-Schmidt on rows a and b, then c = (a x b)^*), so that the third row
 * is exactly the 12-real reconstruction of the first two up to rounding.
 *
 * Layouts (all double, complex stored as re, im):
 *   gauge   U[V][4][3][3][2], V sites lexicographic with x fastest,
 *           mu = 0..3 for x, y, z, t; U[site][mu] is the link site -> site+mu.
 *   spinor  psi[n][4][3][2] for n sites.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  __uint128_t p = (__uint128_t)a * (__uint128_t)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

/* Philox4x64 with 10 rounds: out = philox(ctr, key). */
void wdg_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
  uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(PHILOX_M0, c0, &hi0, &lo0);
    mulhilo64(PHILOX_M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform double in the open interval (0, 1) from the top 53 bits. */
static inline double u01(uint64_t x) {
  return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* Four uniforms for draw (stream, index, block) under seed. */
static inline void draw4(uint64_t seed, uint64_t stream, uint64_t index, uint64_t block,
                         double u[4]) {
  uint64_t ctr[4] = {index, block, stream, 0x5744534c41545449ULL};
  uint64_t key[2] = {seed, 0x0911319100000000ULL};
  uint64_t r[4];
  wdg_philox4x64_10(ctr, key, r);
  for (int i = 0; i < 4; ++i) u[i] = u01(r[i]);
}

/* n Gaussians (n a multiple of 4) for (stream, index), blocks 0, 1, ... */
static void gaussians(uint64_t seed, uint64_t stream, uint64_t index, int n, double *g) {
  const double two_pi = 6.283185307179586476925286766559;
  for (int b = 0; 4 * b < n; ++b) {
    double u[4];
    draw4(seed, stream, index, (uint64_t)b, u);
    for (int k = 0; k < 2; ++k) {
      double rad = sqrt(-2.0 * log(u[2 * k]));
      double ang = two_pi * u[2 * k + 1];
      g[4 * b + 2 * k] = rad * cos(ang);
      g[4 * b + 2 * k + 1] = rad * sin(ang);
    }
  }
}

/* ---- 3x3 complex helpers (row-major, interleaved re/im) ---------------- */
typedef struct { double re, im; } cplx;

static inline cplx cmul(cplx a, cplx b) { cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cplx cconj(cplx a) { cplx r = {a.re, -a.im}; return r; }

static void mat_mul(const cplx *a, const cplx *b, cplx *c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = {0.0, 0.0};
      for (int k = 0; k < 3; ++k) {
        cplx p = cmul(a[3 * i + k], b[3 * k + j]);
        s.re += p.re; s.im += p.im;
      }
      c[3 * i + j] = s;
    }
}

/* Q = i * eps * H for the traceless Hermitian part H of the Gaussian matrix A. */
static void make_generator(const double *g18, double eps, cplx *q) {
  cplx a[9], h[9];
  for (int k = 0; k < 9; ++k) { a[k].re = g18[2 * k]; a[k].im = g18[2 * k + 1]; }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx aij = a[3 * i + j], aji = cconj(a[3 * j + i]);
      h[3 * i + j].re = 0.5 * (aij.re + aji.re);
      h[3 * i + j].im = 0.5 * (aij.im + aji.im);
    }
  double tr = (h[0].re + h[4].re + h[8].re) / 3.0;
  for (int i = 0; i < 3; ++i) { h[4 * i].re -= tr; h[4 * i].im = 0.0; }
  for (int k = 0; k < 9; ++k) { q[k].re = -eps * h[k].im; q[k].im = eps * h[k].re; }
}

/* exp(Q) by Taylor series on Q / 2^s, then s squarings. */
static void mat_exp(const cplx *q, cplx *e) {
  const int s = 6, terms = 14;
  double scale = ldexp(1.0, -s);
  cplx qs[9], term[9], tmp[9];
  for (int k = 0; k < 9; ++k) { qs[k].re = q[k].re * scale; qs[k].im = q[k].im * scale; }
  for (int k = 0; k < 9; ++k) { e[k].re = (k % 4 == 0) ? 1.0 : 0.0; e[k].im = 0.0; term[k] = e[k]; }
  for (int n = 1; n <= terms; ++n) {
    mat_mul(term, qs, tmp);
    for (int k = 0; k < 9; ++k) { term[k].re = tmp[k].re / n; term[k].im = tmp[k].im / n; }
    for (int k = 0; k < 9; ++k) { e[k].re += term[k].re; e[k].im += term[k].im; }
  }
  for (int i = 0; i < s; ++i) {
    mat_mul(e, e, tmp);
    memcpy(e, tmp, sizeof(tmp));
  }
}

/* Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1). */
static void reunitarize(cplx *u) {
  cplx *a = u, *b = u + 3, *c = u + 6;
  double na = 0.0;
  for (int j = 0; j < 3; ++j) na += a[j].re * a[j].re + a[j].im * a[j].im;
  na = 1.0 / sqrt(na);
  for (int j = 0; j < 3; ++j) { a[j].re *= na; a[j].im *= na; }
  cplx d = {0.0, 0.0}; /* <a, b> = sum conj(a) b */
  for (int j = 0; j < 3; ++j) { cplx p = cmul(cconj(a[j]), b[j]); d.re += p.re; d.im += p.im; }
  for (int j = 0; j < 3; ++j) { cplx p = cmul(d, a[j]); b[j].re -= p.re; b[j].im -= p.im; }
  double nb = 0.0;
  for (int j = 0; j < 3; ++j) nb += b[j].re * b[j].re + b[j].im * b[j].im;
  nb = 1.0 / sqrt(nb);
  for (int j = 0; j < 3; ++j) { b[j].re *= nb; b[j].im *= nb; }
  for (int j = 0; j < 3; ++j) {
    int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
    cplx p = cmul(a[j1], b[j2]), m = cmul(a[j2], b[j1]);
    c[j].re = p.re - m.re;
    c[j].im = -(p.im - m.im);
  }
}

static void su3_from_gaussians(const double *g, double eps, double *out18) {
  cplx q[9], u[9];
  make_generator(g, eps, q);
  mat_exp(q, u);
  reunitarize(u);
  for (int k = 0; k < 9; ++k) { out18[2 * k] = u[k].re; out18[2 * k + 1] = u[k].im; }
}

/* Stream tags keep the different kinds of draws apart under one seed. */
#define STREAM_GAUGE 0x4741554745ULL
#define STREAM_SU3 0x5355335f4f4dULL
#define STREAM_SPINOR 0x5350494e4f52ULL
#define STREAM_UNIFORM 0x554e49464fULL

/* Gauge field of V*4 links: U = reunitarized exp(i eps H). */
void wdg_gauge_random(double *U, int64_t nsites, double eps, uint64_t seed) {
  int64_t nlinks = nsites * 4;
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < nlinks; ++l) {
    double g[20];
    gaussians(seed, STREAM_GAUGE, (uint64_t)l, 20, g);
    su3_from_gaussians(g, eps, U + 18 * l);
  }
}

/* n random SU(3) matrices (e.g. a gauge transformation per site). */
void wdg_su3_random(double *W, int64_t n, double eps, uint64_t seed, uint64_t stream) {
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < n; ++l) {
    double g[20];
    gaussians(seed, STREAM_SU3 ^ (stream << 48), (uint64_t)l, 20, g);
    su3_from_gaussians(g, eps, W + 18 * l);
  }
}

/* Complex Gaussian spinors: every one of the 24 reals of a site ~ N(0,1). */
void wdg_spinor_gaussian(double *psi, int64_t nsites, uint64_t seed, uint64_t stream) {
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < nsites; ++s) {
    gaussians(seed, STREAM_SPINOR ^ (stream << 48), (uint64_t)s, 24, psi + 24 * s);
  }
}

/* n uniforms in (0, 1), e.g. the random test vector with entries in [0, 1]. */
void wdg_uniform(double *out, int64_t n, uint64_t seed, uint64_t stream) {
  int64_t nb = (n + 3) / 4;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    double u[4];
    draw4(seed, STREAM_UNIFORM ^ (stream << 48), (uint64_t)b, 0, u);
    for (int k = 0; k < 4; ++k)
      if (4 * b + k < n) out[4 * b + k] = u[k];
  }
}
