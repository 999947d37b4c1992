// Fused BLAS-1 kernels of the BiCGstab and CG iterations (Section 5.1), the
// reliable-update steps (Section 5.3, Algorithm 2) and the finalize pass
// that turns FP64 block partials into the solver's scalars on the device.
//
// Every kernel runs on a grid of (site blocks, right-hand sides); a RHS whose
// mask entry is 0 is skipped.  Per-site arithmetic is in the storage
// precision's arithmetic type (FP32 for FP32 and 16-bit fields, FP64 for
// FP64 fields); every cross-site sum is FP64 (wd_reduce.h).
#include "wd_device.h"
#include "wd_reduce.h"

static_assert(wd::kMaxDot == wd::kMaxDotHost, "partial record size");

namespace wd {

template <typename R>
__device__ __forceinline__ cx<R> cload(const double* sc, int k) {
  return {static_cast<R>(sc[k]), static_cast<R>(sc[k + 1])};
}

__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// ---- BiCGstab ---------------------------------------------------------------------
// p <- r + beta (p - omega v), beta = (rho / rho_prev) (alpha / omega)
template <class S>
__global__ void __launch_bounds__(kBlock) k_bicg_p(int Vh, FieldView p, FieldView r, FieldView v,
                                                   const double* __restrict__ sc,
                                                   const int* __restrict__ mask) {
  using R = typename S::real;
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  const double* s = sc + rhs * SC_COUNT;
  const cx<double> beta = cdiv({s[SC_RHO] , s[SC_RHO + 1]}, {s[SC_RHOP], s[SC_RHOP + 1]}) *
                          cdiv({s[SC_ALPHA], s[SC_ALPHA + 1]}, {s[SC_OMEGA], s[SC_OMEGA + 1]});
  const cx<R> b = {static_cast<R>(beta.re), static_cast<R>(beta.im)};
  const cx<R> w = cload<R>(s, SC_OMEGA);
  Spinor<R> P, Rr, Vv;
  load_spinor<S>(p, rhs, i, P);
  load_spinor<S>(r, rhs, i, Rr);
  load_spinor<S>(v, rhs, i, Vv);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) P.v[a][c] = Rr.v[a][c] + b * (P.v[a][c] - w * Vv.v[a][c]);
  store_spinor<S>(p, rhs, i, P);
}

// r <- r - alpha v   (r becomes s)
template <class S>
__global__ void __launch_bounds__(kBlock) k_bicg_s(int Vh, FieldView r, FieldView v,
                                                   const double* __restrict__ sc,
                                                   const int* __restrict__ mask) {
  using R = typename S::real;
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  const cx<R> al = cload<R>(sc + rhs * SC_COUNT, SC_ALPHA);
  Spinor<R> Rr, Vv;
  load_spinor<S>(r, rhs, i, Rr);
  load_spinor<S>(v, rhs, i, Vv);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) Rr.v[a][c] = Rr.v[a][c] - al * Vv.v[a][c];
  store_spinor<S>(r, rhs, i, Rr);
}

// x <- x + alpha p + omega s;  r <- s - omega t  (s lives in r);
// partials: |r|^2, <r~, r>
template <class S>
__global__ void __launch_bounds__(kBlock) k_bicg_xr(int Vh, FieldView x, FieldView r, FieldView p,
                                                    FieldView t, FieldView rt,
                                                    const double* __restrict__ sc,
                                                    const int* __restrict__ mask,
                                                    double* __restrict__ partials) {
  using R = typename S::real;
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d[3] = {0.0, 0.0, 0.0};
  if (i < Vh) {
    const double* s = sc + rhs * SC_COUNT;
    const cx<R> al = cload<R>(s, SC_ALPHA), om = cload<R>(s, SC_OMEGA);
    Spinor<R> X, Ss, P, T, Rt;
    load_spinor<S>(x, rhs, i, X);
    load_spinor<S>(r, rhs, i, Ss);
    load_spinor<S>(p, rhs, i, P);
    load_spinor<S>(t, rhs, i, T);
    load_spinor<S>(rt, rhs, i, Rt);
    R nn = 0, re = 0, im = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X.v[a][c] = X.v[a][c] + al * P.v[a][c] + om * Ss.v[a][c];
        const cx<R> rn = Ss.v[a][c] - om * T.v[a][c];
        Ss.v[a][c] = rn;
        nn += rn.re * rn.re + rn.im * rn.im;
        const cx<R> q = cmulc(Rt.v[a][c], rn);
        re += q.re;
        im += q.im;
      }
    store_spinor<S>(x, rhs, i, X);
    store_spinor<S>(r, rhs, i, Ss);
    d[0] = nn;
    d[1] = re;
    d[2] = im;
  }
  block_sum_store<3>(d, partials + ((int64_t)rhs * gridDim.x + blockIdx.x) * kMaxDot);
}

// ---- CG on the normal equations ---------------------------------------------------
// x <- x + alpha p;  r <- r - alpha q;  partials: |r|^2
template <class S>
__global__ void __launch_bounds__(kBlock) k_cg_xr(int Vh, FieldView x, FieldView r, FieldView p,
                                                  FieldView q, const double* __restrict__ sc,
                                                  const int* __restrict__ mask,
                                                  double* __restrict__ partials) {
  using R = typename S::real;
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d[1] = {0.0};
  if (i < Vh) {
    const R al = static_cast<R>(sc[rhs * SC_COUNT + SC_ALPHA]);
    Spinor<R> X, Rr, P, Q;
    load_spinor<S>(x, rhs, i, X);
    load_spinor<S>(r, rhs, i, Rr);
    load_spinor<S>(p, rhs, i, P);
    load_spinor<S>(q, rhs, i, Q);
    R nn = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X.v[a][c] = X.v[a][c] + al * P.v[a][c];
        Rr.v[a][c] = Rr.v[a][c] - al * Q.v[a][c];
        nn += Rr.v[a][c].re * Rr.v[a][c].re + Rr.v[a][c].im * Rr.v[a][c].im;
      }
    store_spinor<S>(x, rhs, i, X);
    store_spinor<S>(r, rhs, i, Rr);
    d[0] = nn;
  }
  block_sum_store<1>(d, partials + ((int64_t)rhs * gridDim.x + blockIdx.x) * kMaxDot);
}

// p <- r + beta p
template <class S>
__global__ void __launch_bounds__(kBlock) k_cg_p(int Vh, FieldView p, FieldView r,
                                                 const double* __restrict__ sc,
                                                 const int* __restrict__ mask) {
  using R = typename S::real;
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  const R be = static_cast<R>(sc[rhs * SC_COUNT + SC_BETA]);
  Spinor<R> P, Rr;
  load_spinor<S>(p, rhs, i, P);
  load_spinor<S>(r, rhs, i, Rr);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) P.v[a][c] = Rr.v[a][c] + be * P.v[a][c];
  store_spinor<S>(p, rhs, i, P);
}

// ---- generic field operations -----------------------------------------------------
// dst (precision D) <- src (precision S), re-encoding per site.
template <class D, class S>
__global__ void __launch_bounds__(kBlock) k_convert(int Vh, FieldView dst, FieldView src,
                                                    const int* __restrict__ mask) {
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  Spinor<typename S::real> a;
  load_spinor<S>(src, rhs, i, a);
  Spinor<typename D::real> b;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      b.v[s][c] = {static_cast<typename D::real>(a.v[s][c].re), static_cast<typename D::real>(a.v[s][c].im)};
  store_spinor<D>(dst, rhs, i, b);
}

template <class S>
__global__ void __launch_bounds__(kBlock) k_zero(int Vh, FieldView f, const int* __restrict__ mask) {
  using R = typename S::real;
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  Spinor<R> z;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) z.v[s][c] = {R(0), R(0)};
  store_spinor<S>(f, rhs, i, z);
}

// partials: |f|^2
template <class S>
__global__ void __launch_bounds__(kBlock) k_norm2(int Vh, FieldView f, const int* __restrict__ mask,
                                                  double* __restrict__ partials) {
  using R = typename S::real;
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d[1] = {0.0};
  if (i < Vh) {
    Spinor<R> a;
    load_spinor<S>(f, rhs, i, a);
    R nn = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) nn += a.v[s][c].re * a.v[s][c].re + a.v[s][c].im * a.v[s][c].im;
    d[0] = nn;
  }
  block_sum_store<1>(d, partials + ((int64_t)rhs * gridDim.x + blockIdx.x) * kMaxDot);
}

// ---- reliable update ----------------------------------------------------------------
// x (FP64) <- x + xh (low precision, decoded): the groupwise solution update.
template <class S>
__global__ void __launch_bounds__(kBlock) k_accum(int Vh, FieldView x, FieldView xh,
                                                  const int* __restrict__ mask) {
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  Spinor<double> X;
  Spinor<typename S::real> H;
  load_spinor<SF64>(x, rhs, i, X);
  load_spinor<S>(xh, rhs, i, H);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      X.v[s][c] = X.v[s][c] + cx<double>{static_cast<double>(H.v[s][c].re), static_cast<double>(H.v[s][c].im)};
  store_spinor<SF64>(x, rhs, i, X);
}

// partials: |b|^2 of a canonical full-lattice FP64 array [nrhs][2 Vh][24] read
// as 16-byte pairs in address order: block k sums pairs [24 kBlock k,
// 24 kBlock (k + 1)) of its RHS (the reals of 2 kBlock sites), so a RHS has as
// many records as the other BLAS-1 kernels.
__global__ void __launch_bounds__(kBlock) k_canon_norm2(int Vh, const double* __restrict__ canon,
                                                        double* __restrict__ partials) {
  const int rhs = blockIdx.y;
  const int64_t npair = 24 * (int64_t)Vh;  // 16-byte pairs per RHS
  const double2* src = reinterpret_cast<const double2*>(canon) + (int64_t)rhs * npair;
  const int64_t j0 = (int64_t)blockIdx.x * 24 * kBlock + threadIdx.x;
  double nn = 0.0;
#pragma unroll 4
  for (int k = 0; k < 24; ++k) {
    const int64_t j = j0 + (int64_t)k * kBlock;
    if (j < npair) {
      const double2 v = src[j];
      nn += v.x * v.x + v.y * v.y;
    }
  }
  double d[1] = {nn};
  block_sum_store<1>(d, partials + ((int64_t)rhs * gridDim.x + blockIdx.x) * kMaxDot);
}

// rh <- enc(r64); xh <- 0; partials: |rh|^2, <rt, rh> (has_rt = 0: no rt;
// 1: rt read; 2: rt <- enc(r64) too, the shadow residual of a fresh start).
template <class S>
__global__ void __launch_bounds__(kBlock) k_reencode(int Vh, FieldView rh, FieldView xh, FieldView r64,
                                                     FieldView rt, int has_rt,
                                                     const int* __restrict__ mask,
                                                     double* __restrict__ partials) {
  using R = typename S::real;
  const int rhs = blockIdx.y;
  if (mask && !mask[rhs]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d[3] = {0.0, 0.0, 0.0};
  if (i < Vh) {
    Spinor<double> a;
    load_spinor<SF64>(r64, rhs, i, a);
    Spinor<R> b, z;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        b.v[s][c] = {static_cast<R>(a.v[s][c].re), static_cast<R>(a.v[s][c].im)};
        z.v[s][c] = {R(0), R(0)};
      }
    store_spinor<S>(rh, rhs, i, b);
    if (has_rt == 2) store_spinor<S>(rt, rhs, i, b);
    store_spinor<S>(xh, rhs, i, z);
    // the dots see the stored (re-encoded) residual
    load_spinor<S>(rh, rhs, i, b);
    R nn = 0, re = 0, im = 0;
    Spinor<R> t;
    if (has_rt == 1) load_spinor<S>(rt, rhs, i, t);
    if (has_rt == 2) t = b;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        nn += b.v[s][c].re * b.v[s][c].re + b.v[s][c].im * b.v[s][c].im;
        if (has_rt) {
          const cx<R> q = cmulc(t.v[s][c], b.v[s][c]);
          re += q.re;
          im += q.im;
        }
      }
    d[0] = nn;
    d[1] = re;
    d[2] = im;
  }
  block_sum_store<3>(d, partials + ((int64_t)rhs * gridDim.x + blockIdx.x) * kMaxDot);
}

// ---- finalize: partials -> scalars (one block per RHS) ---------------------------------
struct FinArgs {
  double delta;  // reliable-update trigger (defect correction: inner tolerance)
  double tol;    // target relative residual
  int restart;   // 1: defect correction (Algorithm 1), 0: reliable updates (Algorithm 2)
};

__global__ void __launch_bounds__(kBlock) k_finalize(int stage, int nb, const double* __restrict__ partials,
                                                     double* __restrict__ sc, int* __restrict__ fl,
                                                     int* __restrict__ active, int* __restrict__ rumask,
                                                     const int* __restrict__ mask, FinArgs fa) {
  const int rhs = blockIdx.x;
  if (mask && !mask[rhs]) return;
  double v[4];  // component 3: FIN_TRUE_RHO only (other stages leave it unset)
  sum_partials<4>(partials + (int64_t)rhs * nb * kMaxDot, nb, v);
  if (threadIdx.x != 0) return;
  double* s = sc + rhs * SC_COUNT;
  int* f = fl + rhs * FL_COUNT;
  const double stop = fa.tol * sqrt(s[SC_B2]);
  switch (stage) {
    case FIN_B2: {  // |b|; the solve then runs on b / |b| (B2 becomes 1)
      const double b2 = v[0];
      s[SC_BNORM] = sqrt(b2);
      s[SC_B2] = isfinite(b2) ? (b2 > 0.0 ? 1.0 : 0.0) : b2;
      break;
    }
    case FIN_TRUE: {  // true FP64 residual after a (re)computation of r = b - M x
      s[SC_RTRUE2] = v[0];
      s[SC_MMAX] = sqrt(v[0]);
      f[FL_CONV] = (sqrt(v[0]) <= stop) ? 1 : 0;
      if (!isfinite(v[0])) f[FL_BREAK] = stage + 1;
      // iteration resumes (an RHS that triggered the update was paused) unless done
      active[rhs] = (f[FL_CONV] || f[FL_BREAK]) ? 0 : 1;
      // FL_RU stays as the iteration set it: the host counts the update from it
      rumask[rhs] = active[rhs];  // the residual is re-seeded only where iteration goes on
      break;
    }
    case FIN_RHO: {  // after re-encoding r: rho = <r~, r^>, |r^|^2
      s[SC_R2] = v[0];
      s[SC_RHO] = v[1];
      s[SC_RHO + 1] = v[2];
      break;
    }
    case FIN_TRUE_INIT:   // the same with a new shadow residual: a first iteration follows
    case FIN_TRUE_RHO: {  // both, from the residual dslash that re-encoded r itself
      s[SC_RTRUE2] = v[0];
      s[SC_MMAX] = sqrt(v[0]);
      f[FL_CONV] = (sqrt(v[0]) <= stop) ? 1 : 0;
      if (!isfinite(v[0])) f[FL_BREAK] = FIN_TRUE + 1;
      active[rhs] = (f[FL_CONV] || f[FL_BREAK]) ? 0 : 1;
      rumask[rhs] = active[rhs];
      if (active[rhs]) {
        s[SC_R2] = v[1];
        s[SC_RHO] = v[2];
        s[SC_RHO + 1] = v[3];
        if (stage == FIN_TRUE_INIT) {
          s[SC_RHOP] = 1.0; s[SC_RHOP + 1] = 0.0;
          s[SC_ALPHA] = 1.0; s[SC_ALPHA + 1] = 0.0;
          s[SC_OMEGA] = 1.0; s[SC_OMEGA + 1] = 0.0;
        }
      }
      break;
    }
    case FIN_BICG_INIT: {
      s[SC_R2] = v[0];
      s[SC_RHO] = v[1];
      s[SC_RHO + 1] = v[2];
      s[SC_RHOP] = 1.0; s[SC_RHOP + 1] = 0.0;
      s[SC_ALPHA] = 1.0; s[SC_ALPHA + 1] = 0.0;
      s[SC_OMEGA] = 1.0; s[SC_OMEGA + 1] = 0.0;
      break;
    }
    case FIN_BICG_ALPHA: {  // alpha = rho / <r~, v>
      ++f[FL_ITERS];
      const cx<double> d = {v[0], v[1]};
      if (!(d.re * d.re + d.im * d.im > 0.0) || !isfinite(d.re) || !isfinite(d.im)) {
        f[FL_BREAK] = stage + 1;
        active[rhs] = 0;
        break;
      }
      const cx<double> a = cdiv({s[SC_RHO], s[SC_RHO + 1]}, d);
      s[SC_ALPHA] = a.re;
      s[SC_ALPHA + 1] = a.im;
      break;
    }
    case FIN_BICG_OMEGA: {  // omega = <t, s> / <t, t>
      if (v[2] == 0.0 && v[0] == 0.0 && v[1] == 0.0) {
        // t = M_hat s = 0 means s = 0: the step already solved the system and
        // omega is arbitrary; 1 keeps the next beta finite (r becomes 0 and a
        // reliable update follows)
        s[SC_OMEGA] = 1.0;
        s[SC_OMEGA + 1] = 0.0;
        break;
      }
      if (!(v[2] > 0.0) || !isfinite(v[2])) {
        f[FL_BREAK] = stage + 1;
        active[rhs] = 0;
        break;
      }
      s[SC_OMEGA] = v[0] / v[2];
      s[SC_OMEGA + 1] = v[1] / v[2];
      break;
    }
    case FIN_BICG_ITER: {  // |r^|^2, <r~, r^>; reliable-update trigger
      s[SC_RHOP] = s[SC_RHO];
      s[SC_RHOP + 1] = s[SC_RHO + 1];
      s[SC_RHO] = v[1];
      s[SC_RHO + 1] = v[2];
      s[SC_R2] = v[0];
      const double rn = sqrt(v[0]);
      if (!isfinite(rn) || !(s[SC_OMEGA] * s[SC_OMEGA] + s[SC_OMEGA + 1] * s[SC_OMEGA + 1] > 0.0)) {
        f[FL_BREAK] = stage + 1;
        active[rhs] = 0;
        break;
      }
      // reliable updates: against the largest |r^| since the last update;
      // defect correction: against the residual the inner solve started from
      if (!fa.restart) s[SC_MMAX] = fmax(s[SC_MMAX], rn);
      const int ru = (rn < fa.delta * s[SC_MMAX]) || (rn <= stop);
      f[FL_RU] = ru;
      rumask[rhs] = ru;
      if (ru) active[rhs] = 0;  // paused until the host has run the update
      break;
    }
    case FIN_CG_INIT: {  // rho = |r^|^2 of the normal-equation residual; internal target
      s[SC_R2] = v[0];
      s[SC_RHO] = v[0];
      s[SC_TOLN] = fa.tol * sqrt(v[0]);
      s[SC_MMAX] = sqrt(v[0]);
      break;
    }
    case FIN_CG_ALPHA: {  // alpha = rho / |M p|^2
      ++f[FL_ITERS];
      if (!(v[0] > 0.0) || !isfinite(v[0])) {
        f[FL_BREAK] = stage + 1;
        active[rhs] = 0;
        break;
      }
      s[SC_ALPHA] = s[SC_RHO] / v[0];
      break;
    }
    case FIN_CG_ITER: {  // beta = |r_new|^2 / |r_old|^2; reliable-update trigger
      const double rn = sqrt(v[0]);
      if (!isfinite(rn)) {
        f[FL_BREAK] = stage + 1;
        active[rhs] = 0;
        break;
      }
      s[SC_RHOP] = s[SC_RHO];
      s[SC_RHO] = v[0];
      s[SC_R2] = v[0];
      s[SC_BETA] = v[0] / s[SC_RHOP];
      if (!fa.restart) s[SC_MMAX] = fmax(s[SC_MMAX], rn);
      const int ru = (rn < fa.delta * s[SC_MMAX]) || (rn <= s[SC_TOLN]);
      f[FL_RU] = ru;
      rumask[rhs] = ru;
      if (ru) active[rhs] = 0;  // paused until the host has run the update
      break;
    }
    case FIN_CG_RHO: {  // after a reliable update: new |r^|^2, beta against the old rho
      s[SC_R2] = v[0];
      s[SC_RHO] = v[0];
      s[SC_BETA] = fa.restart ? 0.0 : v[0] / s[SC_RHOP];  // defect correction: p = r^
      s[SC_MMAX] = sqrt(v[0]);
      break;
    }
    default: break;
  }
}

// CG stopping: at a reliable update the true residual |r| of M_hat x = b_hat is
// known; if it misses tol |b| the internal target on the normal-equation
// residual is tightened by the ratio.  Runs after FIN_TRUE.
__global__ void k_cg_tighten(int nrhs, double* sc, const int* fl, const int* mask, double tol) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs || (mask && !mask[rhs])) return;
  double* s = sc + rhs * SC_COUNT;
  if (fl[rhs * FL_COUNT + FL_CONV]) return;
  const double stop = tol * sqrt(s[SC_B2]);
  const double rt = sqrt(s[SC_RTRUE2]);
  if (rt > stop) s[SC_TOLN] = fmin(s[SC_TOLN], s[SC_TOLN] * stop / rt);
}

__global__ void k_init_flags(int nrhs, int* fl, int* active, int* rumask) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  for (int k = 0; k < FL_COUNT; ++k) fl[rhs * FL_COUNT + k] = 0;
  active[rhs] = 1;
  rumask[rhs] = 1;
}

// ---- launchers ----------------------------------------------------------------------------
template <class Fn>
static hipError_t by_prec(wd_prec p, Fn&& fn) {
  switch (p) {
    case WD_FP64: fn(SF64{}); break;
    case WD_FP32: fn(SF32{}); break;
    case WD_HALF_I16: fn(SI16{}); break;
    case WD_HALF_F16: fn(SF16{}); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static FieldView fv(const Field& f) { return FieldView{f.ptr, f.stride, f.nrhs}; }
static dim3 grid_of(const Geom& g, int nrhs) { return dim3((g.Vh + kBlock - 1) / kBlock, nrhs); }

hipError_t blas_bicg_p(const Geom& g, wd_prec pr, Field p, Field r, Field v, const double* sc,
                       const int* mask, hipStream_t s) {
  return by_prec(pr, [&](auto tag) {
    using S = decltype(tag);
    k_bicg_p<S><<<grid_of(g, p.nrhs), kBlock, 0, s>>>(g.Vh, fv(p), fv(r), fv(v), sc, mask);
  });
}

hipError_t blas_bicg_s(const Geom& g, wd_prec pr, Field r, Field v, const double* sc,
                       const int* mask, hipStream_t s) {
  return by_prec(pr, [&](auto tag) {
    using S = decltype(tag);
    k_bicg_s<S><<<grid_of(g, r.nrhs), kBlock, 0, s>>>(g.Vh, fv(r), fv(v), sc, mask);
  });
}

hipError_t blas_bicg_xr(const Geom& g, wd_prec pr, Field x, Field r, Field p, Field t, Field rt,
                        const double* sc, const int* mask, double* partials, hipStream_t s) {
  return by_prec(pr, [&](auto tag) {
    using S = decltype(tag);
    k_bicg_xr<S><<<grid_of(g, x.nrhs), kBlock, 0, s>>>(g.Vh, fv(x), fv(r), fv(p), fv(t), fv(rt), sc,
                                                       mask, partials);
  });
}

hipError_t blas_cg_xr(const Geom& g, wd_prec pr, Field x, Field r, Field p, Field q,
                      const double* sc, const int* mask, double* partials, hipStream_t s) {
  return by_prec(pr, [&](auto tag) {
    using S = decltype(tag);
    k_cg_xr<S><<<grid_of(g, x.nrhs), kBlock, 0, s>>>(g.Vh, fv(x), fv(r), fv(p), fv(q), sc, mask, partials);
  });
}

hipError_t blas_cg_p(const Geom& g, wd_prec pr, Field p, Field r, const double* sc,
                     const int* mask, hipStream_t s) {
  return by_prec(pr, [&](auto tag) {
    using S = decltype(tag);
    k_cg_p<S><<<grid_of(g, p.nrhs), kBlock, 0, s>>>(g.Vh, fv(p), fv(r), sc, mask);
  });
}

hipError_t blas_convert(const Geom& g, wd_prec dst_prec, Field dst, wd_prec src_prec, Field src,
                        const int* mask, hipStream_t s) {
  return by_prec(dst_prec, [&](auto dtag) {
    using D = decltype(dtag);
    (void)by_prec(src_prec, [&](auto stag) {
      using S = decltype(stag);
      k_convert<D, S><<<grid_of(g, dst.nrhs), kBlock, 0, s>>>(g.Vh, fv(dst), fv(src), mask);
    });
  });
}

hipError_t blas_zero(const Geom& g, wd_prec pr, Field f, const int* mask, hipStream_t s) {
  return by_prec(pr, [&](auto tag) {
    using S = decltype(tag);
    k_zero<S><<<grid_of(g, f.nrhs), kBlock, 0, s>>>(g.Vh, fv(f), mask);
  });
}

hipError_t blas_norm2(const Geom& g, wd_prec pr, Field f, const int* mask, double* partials,
                      hipStream_t s) {
  return by_prec(pr, [&](auto tag) {
    using S = decltype(tag);
    k_norm2<S><<<grid_of(g, f.nrhs), kBlock, 0, s>>>(g.Vh, fv(f), mask, partials);
  });
}

hipError_t blas_accum(const Geom& g, wd_prec pr, Field x64, Field xh, const int* mask, hipStream_t s) {
  return by_prec(pr, [&](auto tag) {
    using S = decltype(tag);
    k_accum<S><<<grid_of(g, x64.nrhs), kBlock, 0, s>>>(g.Vh, fv(x64), fv(xh), mask);
  });
}

hipError_t blas_canon_norm2(const Geom& g, const double* canon, int nrhs, double* partials, hipStream_t s) {
  k_canon_norm2<<<grid_of(g, nrhs), kBlock, 0, s>>>(g.Vh, canon, partials);
  return hipGetLastError();
}

hipError_t blas_reencode(const Geom& g, wd_prec pr, Field rh, Field xh, Field r64, const Field* rt,
                         const int* mask, double* partials, hipStream_t s, bool set_rt) {
  if (set_rt && !rt) return hipErrorInvalidValue;
  return by_prec(pr, [&](auto tag) {
    using S = decltype(tag);
    k_reencode<S><<<grid_of(g, rh.nrhs), kBlock, 0, s>>>(g.Vh, fv(rh), fv(xh), fv(r64),
                                                         rt ? fv(*rt) : FieldView{nullptr, 0, 0},
                                                         rt ? (set_rt ? 2 : 1) : 0, mask, partials);
  });
}

hipError_t solver_finalize(int stage, int nrhs, int nb, const double* partials, double* sc, int* fl,
                           int* active, int* rumask, const int* mask, double delta, double tol,
                           int restart, hipStream_t s) {
  k_finalize<<<nrhs, kBlock, 0, s>>>(stage, nb, partials, sc, fl, active, rumask, mask,
                                     FinArgs{delta, tol, restart});
  return hipGetLastError();
}

hipError_t solver_cg_tighten(int nrhs, double* sc, const int* fl, const int* mask, double tol,
                             hipStream_t s) {
  k_cg_tighten<<<(nrhs + 63) / 64, 64, 0, s>>>(nrhs, sc, fl, mask, tol);
  return hipGetLastError();
}

hipError_t solver_init_flags(int nrhs, int* fl, int* active, int* rumask, hipStream_t s) {
  k_init_flags<<<(nrhs + 63) / 64, 64, 0, s>>>(nrhs, fl, active, rumask);
  return hipGetLastError();
}

}  // namespace wd
