/*
 * FP64 CPU oracle for the even-odd preconditioned Wilson-Dirac path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code,
 * header or table with the GPU library, and the GPU library never calls it.
 *
 * Everything is written straight from the paper's formulas, in double
 * precision complex arithmetic, with no spin-projection trick and no link
 * compression:
 *   - Wilson-Dirac matrix and hopping term D (Section 3, Eq. 1).  The hop
 *     x -> x+mu carries (1 - gamma_mu) U_x^mu, the hop x -> x-mu carries
 *     (1 + gamma_mu) (U_{x-mu}^mu)^dagger; both act as a full 4x4 spin
 *     matrix times a full 3x3 colour matrix.
 *   - gamma matrices of the DeGrand-Rossi basis, read off the printed
 *     projectors P^{+-mu} = 1 +- gamma_mu (Appendix B).
 *   - Schur complement on the even sites, M_hat = 1 - kappa^2 D_eo D_oe,
 *     kappa = 1/(2(4+m)) (Section 3, Eq. 2).  The adjoint M_hat^dagger is the
 *     explicit adjoint: conjugate-transposed links, projectors swapped.
 *   - Source preparation and solution reconstruction for the even-odd solve
 *     (the "trivial reconstruction" of Section 3, written out from the
 *     2x2 block form of 1 - kappa D).
 *   - BiCGstab on M_hat and CG on the normal equations M_hat^dag M_hat
 *     (Section 5.1), textbook forms, FP64 throughout.
 *   - The 16-bit storage formats of Section 4.6: a per-site norm (the largest
 *     |component| of the 24 reals) and 24 16-bit numbers per spinor; links
 *     stored as 16-bit numbers in [-1, 1].  The quantisation decisions are
 *     taken in binary32, the precision the GPU kernels take them in.
 *
 * Conventions (readings where the paper is silent):
 *   lattice dims L = (Lx, Ly, Lz, Lt), mu = 0..3 for x, y, z, t (the paper's
 *   mu = 1..4, gamma_4 temporal); site index lex = x + Lx(y + Ly(z + Lz t));
 *   parity (x+y+z+t) mod 2; checkerboard index cb = lex / 2; periodic in x, y,
 *   z; in t periodic or antiperiodic (a hop that crosses the t boundary gets a
 *   factor -1).
 * Layouts (double, complex = re, im):
 *   gauge U[V][4][3][3], full spinor psi[V][4][3], parity spinor psi[Vh][4][3].
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
  int L[4];
  int64_t V, Vh;
  int antiperiodic_t;
} lat_t;

static lat_t make_lat(const int32_t dims[4], int tap) {
  lat_t l;
  l.V = 1;
  for (int m = 0; m < 4; ++m) { l.L[m] = dims[m]; l.V *= dims[m]; }
  l.Vh = l.V / 2;
  l.antiperiodic_t = tap;
  return l;
}

static void coords_of(const lat_t *l, int64_t lex, int x[4]) {
  for (int m = 0; m < 4; ++m) { x[m] = (int)(lex % l->L[m]); lex /= l->L[m]; }
}

static int64_t lex_of(const lat_t *l, const int x[4]) {
  return x[0] + (int64_t)l->L[0] * (x[1] + (int64_t)l->L[1] * (x[2] + (int64_t)l->L[2] * x[3]));
}

static int parity_of(const int x[4]) { return (x[0] + x[1] + x[2] + x[3]) & 1; }

/* lex index of the k-th site (cb index k) of parity p. */
static int64_t lex_of_cb(const lat_t *l, int64_t cb, int p) {
  int64_t lex = 2 * cb;
  int x[4];
  coords_of(l, lex, x);
  if (parity_of(x) != p) lex += 1;
  return lex;
}

/* ---- gamma matrices, DeGrand-Rossi basis (Appendix B) ------------------- */
/* gamma_mu = P^{+mu} - 1 read off the printed projector tables. */
static const cplx GAMMA[4][4][4] = {
    /* gamma_1 (x) */
    {{0, 0, 0, I}, {0, 0, I, 0}, {0, -I, 0, 0}, {-I, 0, 0, 0}},
    /* gamma_2 (y) */
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    /* gamma_3 (z) */
    {{0, 0, I, 0}, {0, 0, 0, -I}, {-I, 0, 0, 0}, {0, I, 0, 0}},
    /* gamma_4 (t) */
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

/* Export gamma_mu as 4x4 complex (re, im interleaved) for the tests. */
void wdo_gamma(int mu, double *out) {
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      out[2 * (4 * a + b)] = creal(GAMMA[mu][a][b]);
      out[2 * (4 * a + b) + 1] = cimag(GAMMA[mu][a][b]);
    }
}

/* ---- hopping term D at one site (Eq. 1) --------------------------------- */
/*
 * out(x) = sum_mu [ (1 - s gamma_mu) U_x^mu psi(x+mu) eta_+(x,mu)
 *                 + (1 + s gamma_mu) U_{x-mu}^mu^dagger psi(x-mu) eta_-(x,mu) ]
 * with s = +1 for D and s = -1 for D^dagger (the adjoint swaps the
 * projectors).  eta = -1 for a t hop across the boundary when antiperiodic.
 * src_parity_layout: src holds only the sites of the opposite parity to x,
 * indexed by cb; otherwise src is a full lattice indexed by lex.
 */
static void hop_site(const lat_t *l, const cplx *U, const cplx *src, int src_parity_layout,
                     int64_t lex_x, int dagger, cplx out[12]) {
  int x[4];
  coords_of(l, lex_x, x);
  const double s = dagger ? -1.0 : 1.0;
  for (int k = 0; k < 12; ++k) out[k] = 0;
  for (int mu = 0; mu < 4; ++mu) {
    for (int dir = 0; dir < 2; ++dir) { /* 0: forward x+mu, 1: backward x-mu */
      int y[4] = {x[0], x[1], x[2], x[3]};
      double eta = 1.0;
      if (dir == 0) {
        y[mu] = x[mu] + 1;
        if (y[mu] == l->L[mu]) { y[mu] = 0; if (mu == 3 && l->antiperiodic_t) eta = -1.0; }
      } else {
        y[mu] = x[mu] - 1;
        if (y[mu] < 0) { y[mu] = l->L[mu] - 1; if (mu == 3 && l->antiperiodic_t) eta = -1.0; }
      }
      int64_t lex_y = lex_of(l, y);
      const cplx *psi = src + 12 * (src_parity_layout ? lex_y / 2 : lex_y);
      /* colour matrix W: U_x^mu forward, (U_{x-mu}^mu)^dagger backward */
      cplx W[3][3];
      if (dir == 0) {
        const cplx *u = U + 9 * (4 * lex_x + mu);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) W[a][b] = u[3 * a + b];
      } else {
        const cplx *u = U + 9 * (4 * lex_y + mu);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) W[a][b] = conj(u[3 * b + a]);
      }
      /* spin matrix S = 1 - s gamma (forward) or 1 + s gamma (backward) */
      double sg = (dir == 0) ? -s : s;
      cplx S[4][4];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) S[a][b] = (a == b ? 1.0 : 0.0) + sg * GAMMA[mu][a][b];
      /* out += eta * (S (x) W) psi */
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) {
          cplx acc = 0;
          for (int b = 0; b < 4; ++b)
            for (int d = 0; d < 3; ++d) acc += S[a][b] * W[c][d] * psi[3 * b + d];
          out[3 * a + c] += eta * acc;
        }
    }
  }
}

/* out = D in on the full lattice (dagger != 0: D^dagger). */
void wdo_dslash_full(const int32_t dims[4], int tap, const double *U, const double *in,
                     double *out, int dagger) {
  lat_t l = make_lat(dims, tap);
#pragma omp parallel for schedule(static)
  for (int64_t lex = 0; lex < l.V; ++lex)
    hop_site(&l, (const cplx *)U, (const cplx *)in, 0, lex, dagger, (cplx *)out + 12 * lex);
}

/* out_p = D_{p,1-p} in_{1-p}: output on the sites of parity p (cb order). */
void wdo_dslash_parity(const int32_t dims[4], int tap, const double *U, const double *in,
                       double *out, int out_parity, int dagger) {
  lat_t l = make_lat(dims, tap);
#pragma omp parallel for schedule(static)
  for (int64_t cb = 0; cb < l.Vh; ++cb) {
    int64_t lex = lex_of_cb(&l, cb, out_parity);
    hop_site(&l, (const cplx *)U, (const cplx *)in, 1, lex, dagger, (cplx *)out + 12 * cb);
  }
}

/* Same as wdo_dslash_parity at n listed output sites (cb indices) only. */
void wdo_dslash_parity_sites(const int32_t dims[4], int tap, const double *U, const double *in,
                             int out_parity, int dagger, const int64_t *cbs, int64_t n,
                             double *out) {
  lat_t l = make_lat(dims, tap);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    int64_t lex = lex_of_cb(&l, cbs[k], out_parity);
    hop_site(&l, (const cplx *)U, (const cplx *)in, 1, lex, dagger, (cplx *)out + 12 * k);
  }
}

/* ---- even-odd operator (Eq. 2) ------------------------------------------ */
/* out_e = (1 - kappa^2 D_eo D_oe) in_e; dagger: the explicit adjoint. */
void wdo_mhat(const int32_t dims[4], int tap, const double *U, double kappa, const double *in,
              double *out, int dagger) {
  lat_t l = make_lat(dims, tap);
  cplx *tmp_o = malloc(sizeof(cplx) * 12 * l.Vh);
  cplx *tmp_e = malloc(sizeof(cplx) * 12 * l.Vh);
  wdo_dslash_parity(dims, tap, U, in, (double *)tmp_o, 1, dagger);
  wdo_dslash_parity(dims, tap, U, (const double *)tmp_o, (double *)tmp_e, 0, dagger);
  const cplx *x = (const cplx *)in;
  cplx *y = (cplx *)out;
  for (int64_t i = 0; i < 12 * l.Vh; ++i) y[i] = x[i] - kappa * kappa * tmp_e[i];
  free(tmp_o);
  free(tmp_e);
}

/* out = (1 - kappa D) in on the full lattice (the kappa-normalised Eq. 1). */
void wdo_mfull(const int32_t dims[4], int tap, const double *U, double kappa, const double *in,
               double *out) {
  lat_t l = make_lat(dims, tap);
  cplx *d = malloc(sizeof(cplx) * 12 * l.V);
  wdo_dslash_full(dims, tap, U, in, (double *)d, 0);
  const cplx *x = (const cplx *)in;
  cplx *y = (cplx *)out;
  for (int64_t i = 0; i < 12 * l.V; ++i) y[i] = x[i] - kappa * d[i];
  free(d);
}

/* Split a full-lattice spinor into its parity parts (cb order). */
void wdo_split(const int32_t dims[4], const double *full, double *even, double *odd) {
  lat_t l = make_lat(dims, 0);
  for (int64_t lex = 0; lex < l.V; ++lex) {
    int x[4];
    coords_of(&l, lex, x);
    double *dst = (parity_of(x) ? odd : even) + 24 * (lex / 2);
    memcpy(dst, full + 24 * lex, 24 * sizeof(double));
  }
}

void wdo_join(const int32_t dims[4], const double *even, const double *odd, double *full) {
  lat_t l = make_lat(dims, 0);
  for (int64_t lex = 0; lex < l.V; ++lex) {
    int x[4];
    coords_of(&l, lex, x);
    const double *src = (parity_of(x) ? odd : even) + 24 * (lex / 2);
    memcpy(full + 24 * lex, src, 24 * sizeof(double));
  }
}

/*
 * With (1 - kappa D) written in blocks [[1, -kappa D_eo], [-kappa D_oe, 1]],
 * the odd row gives x_o = b_o + kappa D_oe x_e, and substituting it in the
 * even row gives M_hat x_e = b_e + kappa D_eo b_o.
 */
void wdo_prepare(const int32_t dims[4], int tap, const double *U, double kappa,
                 const double *b_full, double *bhat_e) {
  lat_t l = make_lat(dims, tap);
  cplx *be = malloc(sizeof(cplx) * 12 * l.Vh), *bo = malloc(sizeof(cplx) * 12 * l.Vh);
  cplx *t = malloc(sizeof(cplx) * 12 * l.Vh);
  wdo_split(dims, b_full, (double *)be, (double *)bo);
  wdo_dslash_parity(dims, tap, U, (const double *)bo, (double *)t, 0, 0);
  cplx *y = (cplx *)bhat_e;
  for (int64_t i = 0; i < 12 * l.Vh; ++i) y[i] = be[i] + kappa * t[i];
  free(be); free(bo); free(t);
}

void wdo_reconstruct(const int32_t dims[4], int tap, const double *U, double kappa,
                     const double *b_full, const double *x_e, double *x_full) {
  lat_t l = make_lat(dims, tap);
  cplx *be = malloc(sizeof(cplx) * 12 * l.Vh), *bo = malloc(sizeof(cplx) * 12 * l.Vh);
  cplx *xo = malloc(sizeof(cplx) * 12 * l.Vh);
  wdo_split(dims, b_full, (double *)be, (double *)bo);
  wdo_dslash_parity(dims, tap, U, x_e, (double *)xo, 1, 0);
  for (int64_t i = 0; i < 12 * l.Vh; ++i) xo[i] = bo[i] + kappa * xo[i];
  wdo_join(dims, x_e, (const double *)xo, x_full);
  free(be); free(bo); free(xo);
}

/* ---- vector helpers ----------------------------------------------------- */
static cplx vdot(const cplx *a, const cplx *b, int64_t n) { /* sum conj(a) b */
  cplx s = 0;
  for (int64_t i = 0; i < n; ++i) s += conj(a[i]) * b[i];
  return s;
}
static double vnorm2(const cplx *a, int64_t n) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
  return s;
}

/* ||b_full - (1 - kappa D) x_full|| / ||b_full|| */
double wdo_true_relres(const int32_t dims[4], int tap, const double *U, double kappa,
                       const double *b_full, const double *x_full) {
  lat_t l = make_lat(dims, tap);
  cplx *mx = malloc(sizeof(cplx) * 12 * l.V);
  wdo_mfull(dims, tap, U, kappa, x_full, (double *)mx);
  const cplx *b = (const cplx *)b_full;
  double rr = 0, bb = vnorm2(b, 12 * l.V);
  for (int64_t i = 0; i < 12 * l.V; ++i) {
    cplx r = b[i] - mx[i];
    rr += creal(r) * creal(r) + cimag(r) * cimag(r);
  }
  free(mx);
  return sqrt(rr / bb);
}

/* ---- solvers (Section 5.1) ----------------------------------------------- */
/* info: [0] iterations, [1] residual replacements, [2] converged flag,
 *       [3] final true relative residual of the full system. */

/* BiCGstab (van der Vorst) on M_hat x_e = b_hat_e, x0 = 0, shadow r~ = r0.
 * Stops when the recursive residual reaches tol ||b||; if the true residual is
 * then still above tol ||b|| it replaces the recursive one and continues. */
void wdo_bicgstab(const int32_t dims[4], int tap, const double *U, double kappa,
                  const double *b_full, double *x_full, double tol, int maxiter, double *info) {
  lat_t l = make_lat(dims, tap);
  int64_t n = 12 * l.Vh;
  cplx *bh = malloc(sizeof(cplx) * n), *x = calloc(n, sizeof(cplx)), *r = malloc(sizeof(cplx) * n);
  cplx *rt = malloc(sizeof(cplx) * n), *p = calloc(n, sizeof(cplx)), *v = calloc(n, sizeof(cplx));
  cplx *s = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
  wdo_prepare(dims, tap, U, kappa, b_full, (double *)bh);
  double bnorm = sqrt(vnorm2((const cplx *)b_full, 12 * l.V));
  double stop = tol * bnorm;
  memcpy(r, bh, sizeof(cplx) * n);
  memcpy(rt, r, sizeof(cplx) * n);
  cplx rho_prev = 1, alpha = 1, omega = 1;
  int it = 0, replacements = 0, converged = 0;
  while (it < maxiter) {
    cplx rho = vdot(rt, r, n);
    cplx beta = (rho / rho_prev) * (alpha / omega);
    for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
    wdo_mhat(dims, tap, U, kappa, (const double *)p, (double *)v, 0);
    alpha = rho / vdot(rt, v, n);
    for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
    wdo_mhat(dims, tap, U, kappa, (const double *)s, (double *)t, 0);
    omega = vdot(t, s, n) / vnorm2(t, n);
    for (int64_t i = 0; i < n; ++i) {
      x[i] += alpha * p[i] + omega * s[i];
      r[i] = s[i] - omega * t[i];
    }
    rho_prev = rho;
    ++it;
    if (sqrt(vnorm2(r, n)) <= stop) {
      wdo_mhat(dims, tap, U, kappa, (const double *)x, (double *)t, 0);
      for (int64_t i = 0; i < n; ++i) r[i] = bh[i] - t[i];
      ++replacements;
      if (sqrt(vnorm2(r, n)) <= stop) { converged = 1; break; }
    }
  }
  wdo_reconstruct(dims, tap, U, kappa, b_full, (const double *)x, x_full);
  info[0] = it; info[1] = replacements; info[2] = converged;
  info[3] = wdo_true_relres(dims, tap, U, kappa, b_full, x_full);
  free(bh); free(x); free(r); free(rt); free(p); free(v); free(s); free(t);
}

/* CG on the normal equations M_hat^dag M_hat x_e = M_hat^dag b_hat_e.
 * The target is the original system: ||b_hat - M_hat x|| <= tol ||b||.  CG
 * runs on its own residual with an internal tolerance that is tightened by
 * the ratio of target to achieved residual whenever it is met early. */
void wdo_cgnr(const int32_t dims[4], int tap, const double *U, double kappa, const double *b_full,
              double *x_full, double tol, int maxiter, double *info) {
  lat_t l = make_lat(dims, tap);
  int64_t n = 12 * l.Vh;
  cplx *bh = malloc(sizeof(cplx) * n), *x = calloc(n, sizeof(cplx)), *r = malloc(sizeof(cplx) * n);
  cplx *p = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n), *w = malloc(sizeof(cplx) * n);
  wdo_prepare(dims, tap, U, kappa, b_full, (double *)bh);
  double bnorm = sqrt(vnorm2((const cplx *)b_full, 12 * l.V));
  double stop = tol * bnorm;
  wdo_mhat(dims, tap, U, kappa, (const double *)bh, (double *)r, 1); /* r = M^dag b_hat */
  double tol_n = tol * sqrt(vnorm2(r, n)); /* tol ||M_hat^dag b_hat|| to start with */
  memcpy(p, r, sizeof(cplx) * n);
  double rr = vnorm2(r, n);
  int it = 0, checks = 0, converged = 0;
  while (it < maxiter) {
    wdo_mhat(dims, tap, U, kappa, (const double *)p, (double *)w, 0);
    wdo_mhat(dims, tap, U, kappa, (const double *)w, (double *)q, 1);
    double alpha = rr / vnorm2(w, n);
    for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    double rr_new = vnorm2(r, n);
    ++it;
    if (sqrt(rr_new) <= tol_n) {
      wdo_mhat(dims, tap, U, kappa, (const double *)x, (double *)w, 0);
      for (int64_t i = 0; i < n; ++i) w[i] = bh[i] - w[i];
      double res = sqrt(vnorm2(w, n));
      ++checks;
      if (res <= stop) { converged = 1; break; }
      tol_n *= stop / res;
    }
    double beta = rr_new / rr;
    for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    rr = rr_new;
  }
  wdo_reconstruct(dims, tap, U, kappa, b_full, (const double *)x, x_full);
  info[0] = it; info[1] = checks; info[2] = converged;
  info[3] = wdo_true_relres(dims, tap, U, kappa, b_full, x_full);
  free(bh); free(x); free(r); free(p); free(q); free(w);
}

/* ---- 16-bit storage formats (Section 4.6) -------------------------------- */
/* IEEE 754 binary32 -> binary16, round to nearest, ties to even. */
static uint16_t f32_to_f16_rne(float f) {
  uint32_t xb;
  memcpy(&xb, &f, 4);
  uint32_t sign = (xb >> 16) & 0x8000u;
  uint32_t ax = xb & 0x7fffffffu;
  if (ax >= 0x7f800000u) return (uint16_t)(sign | 0x7c00u | (ax > 0x7f800000u ? 0x200u : 0u));
  int32_t e = (int32_t)(ax >> 23) - 127;
  uint32_t mant = ax & 0x7fffffu;
  if (e > 15) return (uint16_t)(sign | 0x7c00u);
  if (e >= -14) {
    uint32_t h = ((uint32_t)(e + 15) << 10) | (mant >> 13);
    uint32_t rem = mant & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) h += 1; /* may carry to inf */
    return (uint16_t)(sign | h);
  }
  if (e < -25 || (ax >> 23) == 0) return (uint16_t)sign;
  uint32_t mf = mant | 0x800000u;
  int shift = -(e + 1); /* half subnormal unit is 2^-24 */
  uint32_t q = mf >> shift, rem = mf & ((1u << shift) - 1u), halfway = 1u << (shift - 1);
  if (rem > halfway || (rem == halfway && (q & 1u))) q += 1;
  return (uint16_t)(sign | q);
}

static float f16_to_f32(uint16_t h) {
  uint32_t sign = (uint32_t)(h & 0x8000u) << 16, e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
  float v;
  if (e == 0) v = ldexpf((float)m, -24);
  else if (e == 31) v = m ? NAN : INFINITY;
  else v = ldexpf((float)(m | 0x400u), (int)e - 25);
  uint32_t b;
  memcpy(&b, &v, 4);
  b |= sign;
  memcpy(&v, &b, 4);
  return v;
}

void wdo_f32_to_f16(const float *in, uint16_t *out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = f32_to_f16_rne(in[i]);
}
void wdo_f16_to_f32(const uint16_t *in, float *out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = f16_to_f32(in[i]);
}

/*
 * Spinor: for each of n sites, the 24 reals are rounded to binary32, the norm
 * is the largest magnitude among them, and each real is stored relative to it:
 *   kind 0 (int16 fixed point): q = rint(v * (32767/norm)), |q| <= 32767,
 *                               decoded as q * (norm/32767);
 *   kind 1 (binary16):          h = f16(v * (1/norm)), decoded as h * norm.
 * A site with norm 0, or below 2^-100, stores norm 0 and all zeros.
 */
void wdo_encode_spinor16(int kind, int64_t n, const double *in, uint16_t *q, float *norm) {
  for (int64_t s = 0; s < n; ++s) {
    float v[24], nm = 0.0f;
    for (int i = 0; i < 24; ++i) {
      v[i] = (float)in[24 * s + i];
      nm = fmaxf(nm, fabsf(v[i]));
    }
    /* Reading for tiny sites: a norm below 2^-100 would make 32767/norm or
     * 1/norm overflow binary32, so such a site is stored as zero. */
    if (nm < 0x1p-100f) nm = 0.0f;
    norm[s] = nm;
    if (nm == 0.0f) { for (int i = 0; i < 24; ++i) q[24 * s + i] = 0; continue; }
    if (kind == 0) {
      float scale = 32767.0f / nm;
      for (int i = 0; i < 24; ++i) {
        float r = rintf(v[i] * scale);
        if (r > 32767.0f) r = 32767.0f;
        if (r < -32767.0f) r = -32767.0f;
        q[24 * s + i] = (uint16_t)(int16_t)r;
      }
    } else {
      float scale = 1.0f / nm;
      for (int i = 0; i < 24; ++i) q[24 * s + i] = f32_to_f16_rne(v[i] * scale);
    }
  }
}

void wdo_decode_spinor16(int kind, int64_t n, const uint16_t *q, const float *norm, double *out) {
  for (int64_t s = 0; s < n; ++s) {
    if (kind == 0) {
      float d = norm[s] / 32767.0f;
      for (int i = 0; i < 24; ++i) out[24 * s + i] = (double)((float)(int16_t)q[24 * s + i] * d);
    } else {
      for (int i = 0; i < 24; ++i) out[24 * s + i] = (double)(f16_to_f32(q[24 * s + i]) * norm[s]);
    }
  }
}

/* Link reals (all in [-1, 1]): kind 0 q = rint(u * 32767), decoded as
 * q * (1/32767); kind 1 h = f16(u). */
void wdo_encode_link16(int kind, int64_t n, const double *in, uint16_t *q) {
  for (int64_t i = 0; i < n; ++i) {
    float u = (float)in[i];
    if (kind == 0) {
      float r = rintf(u * 32767.0f);
      if (r > 32767.0f) r = 32767.0f;
      if (r < -32767.0f) r = -32767.0f;
      q[i] = (uint16_t)(int16_t)r;
    } else {
      q[i] = f32_to_f16_rne(u);
    }
  }
}

void wdo_decode_link16(int kind, int64_t n, const uint16_t *q, double *out) {
  for (int64_t i = 0; i < n; ++i)
    out[i] = kind == 0 ? (double)((float)(int16_t)q[i] * (1.0f / 32767.0f)) : (double)f16_to_f32(q[i]);
}

/* ---- 8-real link parametrization (Appendix A.2) --------------------------- */
/*
 * An SU(3) matrix with rows a, b, c is stored as the 8 reals
 *   (Re a2, Im a2, Re a3, Im a3, Re b1, Im b1, arg a1, arg c1)
 * (columns numbered 1..3 as in the paper).  Rebuilding it:
 *   |a1| = sqrt(1 - |a2|^2 - |a3|^2)            (the first row is a unit vector)
 *   |c1| = sqrt(1 - |a1|^2 - |b1|^2)            (so is the first column)
 *   a1, c1 from their moduli and phases
 *   N  = sqrt(|a2|^2 + |a3|^2)
 *   b' = (0, -conj(a3), conj(a2)) / N,  c' = conj(a x b') = (N, -conj(a1) a2 / N, -conj(a1) a3 / N)
 *   b  = p1 b' + p2 c',  c = -conj(p2) b' + conj(p1) c',  p1 = conj(c1) / N,  p2 = b1 / N
 * i.e. an SU(2) rotation of the plane orthogonal to a (b1 = N p2, conj(c1) = N p1).
 * A negative argument of either square root (rounding in low precision) is
 * taken as zero, the paper's stabilisation.  Singular at N = 0 (|a1| = 1).
 */
void wdo_encode_link8(int64_t n, const double *U, double *out) {
  for (int64_t i = 0; i < n; ++i) {
    const cplx *u = (const cplx *)(U + 18 * i);
    double *o = out + 8 * i;
    o[0] = creal(u[1]); o[1] = cimag(u[1]);   /* a2 */
    o[2] = creal(u[2]); o[3] = cimag(u[2]);   /* a3 */
    o[4] = creal(u[3]); o[5] = cimag(u[3]);   /* b1 */
    o[6] = carg(u[0]);                        /* arg a1 */
    o[7] = carg(u[6]);                        /* arg c1 */
  }
}

void wdo_decode_link8(int64_t n, const double *in, double *U) {
  for (int64_t i = 0; i < n; ++i) {
    const double *p = in + 8 * i;
    cplx *u = (cplx *)(U + 18 * i);
    const cplx a2 = p[0] + I * p[1], a3 = p[2] + I * p[3], b1 = p[4] + I * p[5];
    double s = 1.0 - (cabs(a2) * cabs(a2) + cabs(a3) * cabs(a3));
    const double ma1 = s > 0.0 ? sqrt(s) : 0.0;
    const cplx a1 = ma1 * (cos(p[6]) + I * sin(p[6]));
    s = 1.0 - (ma1 * ma1 + cabs(b1) * cabs(b1));
    const double mc1 = s > 0.0 ? sqrt(s) : 0.0;
    const cplx c1 = mc1 * (cos(p[7]) + I * sin(p[7]));
    const double N = sqrt(cabs(a2) * cabs(a2) + cabs(a3) * cabs(a3));
    const cplx bp[3] = {0.0, -conj(a3) / N, conj(a2) / N};
    const cplx cp[3] = {N, -conj(a1) * a2 / N, -conj(a1) * a3 / N};
    const cplx p1 = conj(c1) / N, p2 = b1 / N;
    const cplx a[3] = {a1, a2, a3};
    for (int k = 0; k < 3; ++k) {
      u[k] = a[k];
      u[3 + k] = p1 * bp[k] + p2 * cp[k];
      u[6 + k] = -conj(p2) * bp[k] + conj(p1) * cp[k];
    }
  }
}

/* ---- temporal gauge (the gauge-fixing trick of Section 4.3) --------------- */
/*
 * g(x,0) = 1, g(x,t+1) = g(x,t) U_t(x,t) along every time line; then
 * U'_mu(x) = g(x) U_mu(x) g(x+mu)^dagger.  Every temporal link becomes the
 * unit matrix except on the last time slice, where U'_t(x, Lt-1) is the
 * product of the time line's links (the boundary term).  Spinors transform
 * as psi'(x) = g(x) psi(x), so D[U'] = G D[U] G^dagger.
 */
static void mat_mul(const cplx *A, const cplx *B, cplx *C) {   /* C = A B */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

void wdo_gauge_fix_temporal(const int32_t dims[4], const double *U, double *Uout, double *g) {
  const lat_t l = make_lat(dims, 0);
  const cplx *u = (const cplx *)U;
  cplx *uo = (cplx *)Uout, *G = (cplx *)g;
  const int64_t V3 = (int64_t)l.L[0] * l.L[1] * l.L[2];
  for (int64_t s = 0; s < V3; ++s) {
    cplx *g0 = G + 9 * s;                 /* t = 0: lex = s */
    for (int k = 0; k < 9; ++k) g0[k] = (k % 4 == 0) ? 1.0 : 0.0;
    for (int t = 0; t + 1 < l.L[3]; ++t)
      mat_mul(G + 9 * (s + V3 * t), u + 9 * (4 * (s + V3 * t) + 3), G + 9 * (s + V3 * (t + 1)));
  }
#pragma omp parallel for
  for (int64_t i = 0; i < l.V; ++i) {
    int x[4];
    coords_of(&l, i, x);
    for (int mu = 0; mu < 4; ++mu) {
      int y[4] = {x[0], x[1], x[2], x[3]};
      y[mu] = (y[mu] + 1) % l.L[mu];
      const cplx *gx = G + 9 * i, *gy = G + 9 * lex_of(&l, y);
      cplx tmp[9], gyd[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) gyd[3 * a + b] = conj(gy[3 * b + a]);
      mat_mul(gx, u + 9 * (4 * i + mu), tmp);
      mat_mul(tmp, gyd, uo + 9 * (4 * i + mu));
    }
  }
}

/* psi'(x) = g(x) psi(x) (adjoint != 0: g(x)^dagger psi(x)), full lattice, nrhs fields. */
void wdo_gauge_rotate_spinor(const int32_t dims[4], const double *g, const double *in, double *out,
                             int nrhs, int adjoint) {
  const lat_t l = make_lat(dims, 0);
  const cplx *G = (const cplx *)g;
  for (int r = 0; r < nrhs; ++r) {
    const cplx *src = (const cplx *)in + (int64_t)r * l.V * 12;
    cplx *dst = (cplx *)out + (int64_t)r * l.V * 12;
#pragma omp parallel for
    for (int64_t i = 0; i < l.V; ++i)
      for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
          cplx acc = 0.0;
          for (int b = 0; b < 3; ++b) {
            const cplx m = adjoint ? conj(G[9 * i + 3 * b + a]) : G[9 * i + 3 * a + b];
            acc += m * src[12 * i + 3 * s + b];
          }
          dst[12 * i + 3 * s + a] = acc;
        }
  }
}
