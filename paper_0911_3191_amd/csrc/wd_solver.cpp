// Solver drivers: BiCGstab on M_hat and CG on M_hat^dag M_hat (Section 5.1)
// with reliable updates (Section 5.3, Algorithm 2): the Krylov iteration runs
// with its vectors and its M_hat in the inner storage precision; whenever the
// iterated residual has dropped by delta against its maximum since the last
// update (or reaches the target), the inner solution is added to the FP64
// accumulator, the FP64 residual b_hat - M_hat x is recomputed with the FP64
// gauge field and replaces the iterated one, and the inner solution restarts
// from zero.  The Krylov recurrences (p, v, rho, alpha, omega) are kept.
//
// All scalars live in device memory and are produced by finalize kernels, so
// the host only reads a few flags per iteration (reliable-update trigger,
// convergence, breakdown).  The iteration body can be captured once into a
// hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "wd_internal.h"

namespace wd {

static size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// Workspace layout shared by wd_solve_workspace_bytes and the drivers.
struct Layout {
  size_t hi_field, lo_field;
  int n_hi_even, n_hi_odd, n_lo_even, n_lo_odd;
  size_t partials, scalars, flags, masks;
  size_t total;
};

static Layout layout(const Geom& g, int kind, wd_prec inner, int nrhs) {
  Layout L;
  L.hi_field = align256(spinor_field_bytes(g, WD_FP64, nrhs));
  L.lo_field = align256(spinor_field_bytes(g, inner, nrhs));
  // high precision: b_hat, x, r (+ the normal-equation residual for CG with an FP64 inner
  // solver; with a 32- or 16-bit one it goes straight into r^) and an odd temporary
  L.n_hi_even = (kind == WD_SOLVER_CG && inner == WD_FP64) ? 4 : 3;
  L.n_hi_odd = 1;
  // low precision: BiCGstab r^, r~, p, v, t, x^; CG r^, p, q, w, x^; plus an odd temporary
  L.n_lo_even = (kind == WD_SOLVER_CG) ? 5 : 6;
  L.n_lo_odd = 1;
  const int nb = std::max((g.Vh + 255) / 256, dslash_partial_blocks(g, nrhs, LaunchCfg{1, 256}));
  L.partials = align256(sizeof(double) * kMaxDotHost * nb * (size_t)nrhs);
  L.scalars = align256(sizeof(double) * SC_COUNT * (size_t)nrhs);
  L.flags = align256(sizeof(int) * FL_COUNT * (size_t)nrhs);
  L.masks = align256(sizeof(int) * 3 * (size_t)nrhs);  // active, rumask, the list of updating RHS
  L.total = (L.n_hi_even + L.n_hi_odd) * L.hi_field + (L.n_lo_even + L.n_lo_odd) * L.lo_field +
            L.partials + L.scalars + L.flags + L.masks;
  return L;
}

}  // namespace wd

struct wd_solver {
  int kind;
  const wd_gauge* g;
  wd::Geom geom;
  double kappa;
  wd_solve_params prm;
  hipStream_t s;
  double* x_out;
  const double* b_in;
  int nrhs, nb, nb_dslash;  // partial records per RHS: BLAS-1 kernels, fused-dot dslash
  wd::Field bhat, x, r, rn, to64;
  wd::Field rh, rt, p, v, t, xh, to;  // CG uses v as q and t as w; rt unused
  double* partials;
  double* sc;
  int* fl;
  int* active;
  int* rumask;
  int* rumap;      // the RHS of a reliable update, listed (device)
  int* h_fl;       // pinned host copy of the flags
  int* h_map;      // pinned host staging of rumap (after the flags in the same buffer)
  double* h_sc;    // pinned host copy of the scalars
  std::vector<int> iters, rus, status, done_rhs;
  std::string note;  // breakdown details for wd_last_error
  int per_check;     // inner iterations launched between two reads of the flags
  int loops;
  bool finished;
  hipGraph_t graph;
  hipGraphExec_t gexec;
  bool graph_ready;
  std::chrono::steady_clock::time_point t0;
};

namespace wd {

// With n_map > 0 the launch covers only the n_map RHS listed in h->rumap (the
// same set as mask), packed into as few RHS groups as they fill.
static hipError_t dslash_into(wd_solver* h, wd_prec prec, const Field& out, const Field& in,
                              int parity, int dagger, const Field* xpay, double a, int dot,
                              const Field* y, const int* mask, int n_map = 0) {
  DslashArgs d;
  d.out = out;
  d.in = in;
  d.out_parity = parity;
  d.dagger = dagger;
  d.xpay = xpay;
  d.a = a;
  d.dot = dot;
  d.y = y;
  d.partials = h->partials;
  d.active = mask;
  d.basis = kBasisUK;
  if (n_map > 0) {
    d.rhs_map = h->rumap;
    d.n_map = n_map;
  }
  return launch_dslash_ex(h->g, prec, d, h->s);
}

// out_e = in_e - kappa^2 D_eo D_oe in_e (dagger: the adjoint), optional fused dot.
static hipError_t mhat_into(wd_solver* h, wd_prec prec, const Field& out, const Field& in,
                            const Field& tmp_odd, int dagger, int dot, const Field* y,
                            const int* mask, int n_map = 0) {
  hipError_t e = dslash_into(h, prec, tmp_odd, in, 1, dagger, nullptr, 0.0, DOT_NONE, nullptr, mask, n_map);
  if (e != hipSuccess) return e;
  return dslash_into(h, prec, out, tmp_odd, 0, dagger, &in, -h->kappa * h->kappa, dot, y, mask, n_map);
}

// after_dslash: the partial records come from a dslash with a fused dot
// (its record count per RHS), else from a BLAS-1 kernel.
static hipError_t fin(wd_solver* h, int stage, const int* mask, bool after_dslash) {
  return solver_finalize(stage, h->nrhs, after_dslash ? h->nb_dslash : h->nb, h->partials, h->sc,
                         h->fl, h->active, h->rumask, mask, h->prm.delta, h->prm.tol, h->prm.restart,
                         h->s);
}

#define WD_TRY(expr)                         \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

// Tunes the launch shapes of the inner-precision dslash forms of
// iteration_body (each key once per process; see wd_tune.cpp).  Every
// tuning launch reads zeros: p and v are zero after prepare, and the odd
// temporary and t are zeroed here first, so the launches write zeros into
// the odd temporary, v and t whichever keys are already cached (an
// iteration writes those before it reads them, and reads v only times
// beta = 0 in its first p-update, which a stale NaN would poison).
static hipError_t pretune_inner(wd_solver* h) {
  const wd_prec P = h->prm.inner;
  WD_TRY(blas_zero(h->geom, P, h->to, nullptr, h->s));
  WD_TRY(blas_zero(h->geom, P, h->t, nullptr, h->s));
  auto form = [&](const Field& out, const Field& in, int parity, int dagger, const Field* xpay, int dot,
                  const Field* y) {
    DslashArgs d;
    d.out = out;
    d.in = in;
    d.out_parity = parity;
    d.dagger = dagger;
    d.xpay = xpay;
    d.a = -h->kappa * h->kappa;
    d.dot = dot;
    d.y = y;
    d.partials = h->partials;
    d.basis = kBasisUK;
    tune_dslash(h->g, P, d, h->s);
  };
  form(h->to, h->p, 1, 0, nullptr, DOT_NONE, nullptr);  // first half of M_hat p
  if (h->kind == WD_SOLVER_BICGSTAB) {
    form(h->v, h->to, 0, 0, &h->p, DOT_YO, &h->rt);
    form(h->t, h->to, 0, 0, &h->p, DOT_OX, nullptr);
  } else {
    form(h->t, h->to, 0, 0, &h->p, DOT_OO, nullptr);
    form(h->to, h->t, 1, 1, nullptr, DOT_NONE, nullptr);
    form(h->v, h->to, 0, 1, &h->t, DOT_NONE, nullptr);
  }
  return hipSuccess;  // a candidate that fails to launch is skipped by the tuner
}

// One Krylov iteration in the inner precision, all active RHS.
static hipError_t iteration_body(wd_solver* h) {
  const Geom& g = h->geom;
  const wd_prec P = h->prm.inner;
  const int* act = h->active;
  if (h->kind == WD_SOLVER_BICGSTAB) {
    WD_TRY(blas_bicg_p(g, P, h->p, h->rh, h->v, h->sc, act, h->s));
    WD_TRY(mhat_into(h, P, h->v, h->p, h->to, 0, DOT_YO, &h->rt, act));  // v = M p, <r~, v>
    WD_TRY(fin(h, FIN_BICG_ALPHA, act, true));
    WD_TRY(blas_bicg_s(g, P, h->rh, h->v, h->sc, act, h->s));           // s = r - alpha v
    WD_TRY(mhat_into(h, P, h->t, h->rh, h->to, 0, DOT_OX, nullptr, act));  // t = M s, <t,s>, |t|^2
    WD_TRY(fin(h, FIN_BICG_OMEGA, act, true));
    WD_TRY(blas_bicg_xr(g, P, h->xh, h->rh, h->p, h->t, h->rt, h->sc, act, h->partials, h->s));
    WD_TRY(fin(h, FIN_BICG_ITER, act, false));
  } else {
    // w = M p (|w|^2), q = M^dag w, x^ += alpha p, r^ -= alpha q
    WD_TRY(mhat_into(h, P, h->t, h->p, h->to, 0, DOT_OO, nullptr, act));
    WD_TRY(fin(h, FIN_CG_ALPHA, act, true));
    WD_TRY(mhat_into(h, P, h->v, h->t, h->to, 1, DOT_NONE, nullptr, act));
    WD_TRY(blas_cg_xr(g, P, h->xh, h->rh, h->p, h->v, h->sc, act, h->partials, h->s));
    WD_TRY(fin(h, FIN_CG_ITER, act, false));
    // p = r^ + beta p where iteration goes on; an RHS that triggered a
    // reliable update is paused and takes this step after the update
    WD_TRY(blas_cg_p(g, P, h->p, h->rh, h->sc, act, h->s));
  }
  return hipSuccess;
}

// FP64 r = b_hat - M_hat x for the RHS in mask (all when null), then the
// convergence test.  The subtraction from b_hat and |r|^2 are fused into the
// second dslash.  With n_map > 0 the dslash launches cover only the n_map RHS
// listed in h->rumap (the same set as mask), packed into as few RHS groups as
// they fill, rather than the whole batch with most of it masked off.  With
// reencode (BiCGstab with reliable updates) the second dslash does not store
// r in FP64 but re-encodes it into r^ itself, zeroes x^ and returns
// <r~, r^> and |r^|^2 beside |r|^2: the whole re-seed of the inner solver.
// With restart (defect correction) the same pass also writes the new shadow
// residual r~ = r^, and the scalars are those of a first iteration.
static hipError_t true_residual(wd_solver* h, const int* mask, int n_map = 0, bool reencode = false) {
  DslashArgs d;
  d.out = h->to64;
  d.in = h->x;
  d.out_parity = 1;
  d.partials = h->partials;
  d.active = mask;
  d.basis = kBasisUK;
  if (n_map > 0) {
    d.rhs_map = h->rumap;
    d.n_map = n_map;
  }
  WD_TRY(launch_dslash_ex(h->g, WD_FP64, d, h->s));
  d.out = h->r;
  d.in = h->to64;
  d.out_parity = 0;
  d.xpay = &h->x;
  d.a = -h->kappa * h->kappa;
  d.dot = reencode ? DOT_RES_ENC : DOT_RES;
  d.y = &h->bhat;
  d.enc_prec = h->prm.inner;
  d.enc_rh = &h->rh;
  d.enc_xh = &h->xh;
  d.enc_rt = &h->rt;
  d.enc_set_rt = h->prm.restart;
  WD_TRY(launch_dslash_ex(h->g, WD_FP64, d, h->s));
  WD_TRY(fin(h, !reencode ? FIN_TRUE : (h->prm.restart ? FIN_TRUE_INIT : FIN_TRUE_RHO), mask, true));
  if (reencode && h->prm.restart) {  // p = v = 0 where the restarted solve goes on
    WD_TRY(blas_zero(h->geom, h->prm.inner, h->p, h->rumask, h->s));
    WD_TRY(blas_zero(h->geom, h->prm.inner, h->v, h->rumask, h->s));
  }
  return hipSuccess;
}

// Re-seed the inner residual from the FP64 one r64 (and zero x^) for the RHS
// in rumask.  Defect correction restarts BiCGstab there: new shadow residual,
// p = v = 0 and the scalars of a first iteration.  (CG restarts through
// beta = 0 at FIN_CG_RHO, so that the p update after the step sets p = r^.)
// n_map: as for true_residual (CG's M_hat^dag r launches).
static hipError_t reseed(wd_solver* h, bool first, const Field& r64, int n_map = 0) {
  const Geom& g = h->geom;
  const wd_prec P = h->prm.inner;
  if (h->kind == WD_SOLVER_BICGSTAB) {
    const bool fresh = first || h->prm.restart;  // then also r~ = r^
    if (!first && h->prm.restart) {
      WD_TRY(blas_zero(g, P, h->p, h->rumask, h->s));
      WD_TRY(blas_zero(g, P, h->v, h->rumask, h->s));
    }
    WD_TRY(blas_reencode(g, P, h->rh, h->xh, r64, &h->rt, h->rumask, h->partials, h->s, fresh));
    WD_TRY(fin(h, fresh ? FIN_BICG_INIT : FIN_RHO, h->rumask, false));
  } else {
    if (!first) WD_TRY(solver_cg_tighten(h->nrhs, h->sc, h->fl, h->rumask, h->prm.tol, h->s));
    // normal-equation residual M_hat^dag r; r^ = it, x^ = 0.  With a 32- or
    // 16-bit inner format the second FP64 dslash encodes it straight into r^
    // and sums |r^|^2 of the stored values: it is never stored in FP64, and
    // that launch's output names no memory (its shape only sizes the launch).
    const bool fused = P != WD_FP64;
    if (!fused) {
      WD_TRY(mhat_into(h, WD_FP64, h->rn, r64, h->to64, 1, DOT_NONE, nullptr, h->rumask, n_map));
      WD_TRY(blas_reencode(g, P, h->rh, h->xh, h->rn, nullptr, h->rumask, h->partials, h->s));
    } else {
      WD_TRY(dslash_into(h, WD_FP64, h->to64, r64, 1, 1, nullptr, 0.0, DOT_NONE, nullptr, h->rumask, n_map));
      DslashArgs d;
      d.out = Field{nullptr, h->geom.stride, h->nrhs};  // not written
      d.in = h->to64;
      d.out_parity = 0;
      d.dagger = 1;
      d.xpay = &r64;
      d.a = -h->kappa * h->kappa;
      d.dot = DOT_ENC;
      d.partials = h->partials;
      d.active = h->rumask;
      d.basis = kBasisUK;
      d.enc_prec = P;
      d.enc_rh = &h->rh;
      d.enc_xh = &h->xh;
      if (n_map > 0) {
        d.rhs_map = h->rumap;
        d.n_map = n_map;
      }
      WD_TRY(launch_dslash_ex(h->g, WD_FP64, d, h->s));
    }
    WD_TRY(fin(h, first ? FIN_CG_INIT : FIN_CG_RHO, h->rumask, fused));
    if (first) WD_TRY(blas_convert(g, P, h->p, P, h->rh, h->rumask, h->s));  // p = r^
  }
  return hipSuccess;
}

// Mixed-precision BiCGstab re-seeds r^ inside the FP64 dslash, so it never
// writes the FP64 r after prepare, which therefore keeps b_o / |b| there for
// the reconstruction.
static bool fused_reseed(const wd_solver* h) {
  return h->kind == WD_SOLVER_BICGSTAB && h->prm.inner != WD_FP64;
}

static hipError_t reliable_update(wd_solver* h) {
  // the RHS that flagged an update (the device's rumask), listed for the dslash
  int n = 0;
  for (int k = 0; k < h->nrhs; ++k)
    if (!h->done_rhs[k] && h->h_fl[k * FL_COUNT + FL_RU]) h->h_map[n++] = k;
  if (n > 0 && n < h->nrhs)
    WD_TRY(hipMemcpyAsync(h->rumap, h->h_map, sizeof(int) * n, hipMemcpyHostToDevice, h->s));
  else
    n = 0;  // every RHS (or, defensively, none listed): the mask alone
  WD_TRY(blas_accum(h->geom, h->prm.inner, h->x, h->xh, h->rumask, h->s));  // x += x^
  if (fused_reseed(h)) return true_residual(h, h->rumask, n, true);  // r = b - M x; r^ = r, x^ = 0 in the same pass
  WD_TRY(true_residual(h, h->rumask, n));  // r = b - M x
  WD_TRY(reseed(h, false, h->r, n));       // r^ = r (CG: M_hat^dag r), x^ = 0
  return hipSuccess;
}

static const char* const kStageNames[] = {"b2", "b2+", "true residual", "rho", "bicg init",
                                          "alpha", "omega", "bicg iter", "cg init", "cg alpha",
                                          "cg iter", "cg rho"};

static void note_breakdown(wd_solver* h, int k) {
  const int st = h->h_fl[k * FL_COUNT + FL_BREAK] - 1;
  const char* name = (st >= 0 && st < 12) ? kStageNames[st] : "?";
  char buf[160];
  snprintf(buf, sizeof(buf), " rhs %d at %s (iteration %d, |r^|^2 %.3e, rho %.3e)", k, name,
           h->iters[k], h->h_sc[k * SC_COUNT + SC_R2], h->h_sc[k * SC_COUNT + SC_RHO]);
  h->note += buf;
}

static hipError_t read_flags(wd_solver* h) {
  WD_TRY(hipMemcpyAsync(h->h_fl, h->fl, sizeof(int) * FL_COUNT * h->nrhs, hipMemcpyDeviceToHost, h->s));
  WD_TRY(hipMemcpyAsync(h->h_sc, h->sc, sizeof(double) * SC_COUNT * h->nrhs, hipMemcpyDeviceToHost, h->s));
  return hipStreamSynchronize(h->s);
}

static hipError_t prepare(wd_solver* h) {
  const Geom& g = h->geom;
  const int n = h->nrhs;
  WD_TRY(solver_init_flags(n, h->fl, h->active, h->rumask, h->s));
  // |b| of the caller's source, then the solve runs on b / |b| (a unit source
  // per RHS; x is scaled back when it is decoded)
  WD_TRY(blas_canon_norm2(g, h->b_in, h->nrhs, h->partials, h->s));
  WD_TRY(fin(h, FIN_B2, nullptr, false));
  // b_e / |b| -> to64 and b_o / |b| -> r (held there for the reconstruction
  // where the solve leaves r alone; fields hold either parity), rotated into
  // the UKQCD basis every solver field uses (S is orthogonal: norms and inner
  // products are those of the caller's basis)
  WD_TRY(launch_spinor_encode_both(g, h->to64, h->r, h->b_in, h->s, kBasisUK, h->sc, 1));
  // b_hat = b_e + kappa D_eo b_o, with |b_hat|^2 from the same launch.  x = 0,
  // so r = b_hat - M_hat x is b_hat exactly: the convergence test and the
  // first inner residual read b_hat (no further dslash needed)
  WD_TRY(dslash_into(h, WD_FP64, h->bhat, h->r, 0, 0, &h->to64, h->kappa, DOT_OO, nullptr, nullptr));
  WD_TRY(fin(h, FIN_TRUE, nullptr, true));
  WD_TRY(blas_zero(g, WD_FP64, h->x, nullptr, h->s));
  WD_TRY(blas_zero(g, h->prm.inner, h->p, nullptr, h->s));
  WD_TRY(blas_zero(g, h->prm.inner, h->v, nullptr, h->s));
  WD_TRY(reseed(h, true, h->bhat));
  return hipSuccess;
}

// x_o = b_o + kappa D_oe x_e for the unit source (b_o / |b| from r where the
// solve kept it, else encoded again into to64), then both parities into the
// caller's x, times |b| and back in the DeGrand-Rossi basis.
static hipError_t reconstruct(wd_solver* h) {
  const Geom& g = h->geom;
  const Field* bo = &h->r;
  if (!fused_reseed(h)) {
    WD_TRY(launch_spinor_encode_map(g, WD_FP64, h->to64, h->b_in, 1, h->s, kBasisUK, h->sc, 1));
    bo = &h->to64;
  }
  WD_TRY(dslash_into(h, WD_FP64, h->to64, h->x, 1, 0, bo, h->kappa, DOT_NONE, nullptr, nullptr));
  WD_TRY(launch_spinor_decode_both(g, h->x_out, h->x, h->to64, h->s, kBasisUK, h->sc, 2));
  return hipStreamSynchronize(h->s);
}

static wd_status hip_fail(hipError_t e, const char* where) {
  return fail(WD_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace wd

using namespace wd;

namespace {

wd_status validate(int kind, const wd_gauge* g, double kappa, const void* x, const void* b,
                   const wd_solve_params* prm, const void* ws, size_t ws_bytes) {
  if (kind != WD_SOLVER_BICGSTAB && kind != WD_SOLVER_CG) return fail(WD_EINVAL, "unknown solver");
  if (!prm) return fail(WD_EINVAL, "params is NULL");
  if (!std::isfinite(kappa) || kappa <= 0) return fail(WD_EINVAL, "kappa must be finite and > 0");
  if (!(prm->tol > 0) || !std::isfinite(prm->tol)) return fail(WD_EINVAL, "tol must be finite and > 0");
  if (prm->maxiter < 1) return fail(WD_EINVAL, "maxiter must be >= 1");
  if (!(prm->delta >= 0.0 && prm->delta < 1.0)) return fail(WD_EINVAL, "delta must satisfy 0 <= delta < 1");
  if (prm->nrhs < 1 || prm->nrhs > 64) return fail(WD_EINVAL, "nrhs must be in [1, 64]");
  if (prm->inner < WD_FP64 || prm->inner > WD_HALF_F16) return fail(WD_EINVAL, "unknown inner precision");
  if (prm->x0_given != 0) return fail(WD_EUNSUPPORTED, "x0_given is not supported");
  if (prm->check_every < 0 || prm->check_every > 64) return fail(WD_EINVAL, "check_every must be in [0, 64]");
  if (prm->restart < 0 || prm->restart > 1) return fail(WD_EINVAL, "restart must be 0 or 1");
  if (prm->restart == 1 && !(prm->delta > 0.0))
    return fail(WD_EINVAL, "defect correction needs an inner tolerance delta > 0");
  if (!g) return fail(WD_EINVAL, "gauge handle is NULL");
  if (!(g->mask & WD_PREC_MASK(WD_FP64)) || !(g->mask & WD_PREC_MASK(prm->inner)))
    return fail(WD_EINVAL, "gauge handle must hold FP64 and the inner precision");
  for (const void* p : {x, b, ws}) {
    if (!p) return fail(WD_EINVAL, "x, b and workspace must be non-NULL");
    if (reinterpret_cast<uintptr_t>(p) % 256) return fail(WD_EINVAL, "x, b and workspace must be 256-byte aligned");
  }
  if (x == b) return fail(WD_EINVAL, "x and b must not alias");
  const Layout L = layout(g->geom, kind, prm->inner, prm->nrhs);
  if (ws_bytes < L.total)
    return fail(WD_EINVAL, "workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(L.total));
  return WD_OK;
}

double flops_per_iter(int kind) { return kind == WD_SOLVER_CG ? 5616.0 : 6336.0; }
double flops_per_update(int kind) { return kind == WD_SOLVER_CG ? 5616.0 : 2784.0; }

}  // namespace

extern "C" {

size_t wd_solve_workspace_bytes(const wd_lattice* lat, const wd_solve_params* prm, int32_t solver) {
  if (!lat || !prm || (solver != WD_SOLVER_BICGSTAB && solver != WD_SOLVER_CG)) return 0;
  if (wd_gauge_bytes(lat, 1) == 0) return 0;
  if (prm->nrhs < 1 || prm->nrhs > 64 || prm->inner < WD_FP64 || prm->inner > WD_HALF_F16) return 0;
  return layout(make_geom(*lat), solver, prm->inner, prm->nrhs).total;
}

wd_status wd_solver_begin(int32_t solver, const wd_gauge* g, double kappa, double* x, const double* b,
                          const wd_solve_params* prm, void* workspace, size_t ws_bytes, void* stream,
                          wd_solver** out) {
  set_error("");
  if (!out) return fail(WD_EINVAL, "out is NULL");
  *out = nullptr;
  wd_status st = validate(solver, g, kappa, x, b, prm, workspace, ws_bytes);
  if (st) return st;
  wd_solver* h = new (std::nothrow) wd_solver();
  if (!h) return fail(WD_ENOMEM, "host allocation failed");
  h->kind = solver;
  h->g = g;
  h->geom = g->geom;
  h->kappa = kappa;
  h->prm = *prm;
  h->s = static_cast<hipStream_t>(stream);
  h->x_out = x;
  h->b_in = b;
  h->nrhs = prm->nrhs;
  h->nb = (h->geom.Vh + 255) / 256;
  h->nb_dslash = dslash_partial_blocks(h->geom, h->nrhs, LaunchCfg{1, 256});
  const Layout L = layout(h->geom, solver, prm->inner, prm->nrhs);
  char* p = static_cast<char*>(workspace);
  auto take_hi = [&]() { Field f{p, h->geom.stride, h->nrhs}; p += L.hi_field; return f; };
  auto take_lo = [&]() { Field f{p, h->geom.stride, h->nrhs}; p += L.lo_field; return f; };
  h->bhat = take_hi();
  h->x = take_hi();
  h->r = take_hi();
  h->rn = (solver == WD_SOLVER_CG && prm->inner == WD_FP64) ? take_hi() : Field{nullptr, 0, 0};
  h->to64 = take_hi();
  h->rh = take_lo();
  h->p = take_lo();
  h->v = take_lo();
  h->t = take_lo();
  h->xh = take_lo();
  h->rt = (solver == WD_SOLVER_BICGSTAB) ? take_lo() : Field{nullptr, 0, 0};
  h->to = take_lo();
  h->partials = reinterpret_cast<double*>(p);
  p += L.partials;
  h->sc = reinterpret_cast<double*>(p);
  p += L.scalars;
  h->fl = reinterpret_cast<int*>(p);
  p += L.flags;
  h->active = reinterpret_cast<int*>(p);
  h->rumask = h->active + h->nrhs;
  h->rumap = h->rumask + h->nrhs;
  h->iters.assign(h->nrhs, 0);
  h->rus.assign(h->nrhs, 0);
  h->status.assign(h->nrhs, WD_NOT_CONVERGED);
  h->done_rhs.assign(h->nrhs, 0);
  h->graph_ready = false;
  h->finished = false;
  h->per_check = prm->check_every > 1 ? prm->check_every : 1;
  h->loops = 0;
  h->t0 = std::chrono::steady_clock::now();
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->h_fl), sizeof(int) * (FL_COUNT + 1) * h->nrhs);
  h->h_map = h->h_fl + FL_COUNT * h->nrhs;
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&h->h_sc), sizeof(double) * SC_COUNT * h->nrhs);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "pinned host buffer");
  }
  e = prepare(h);  // its FP64 dslash launches pick their own launch shape
  // pick the inner-precision launch shapes of every form an iteration uses
  // before any graph capture
  if (e == hipSuccess) e = pretune_inner(h);
  if (e == hipSuccess) e = read_flags(h);
  if (e != hipSuccess) {
    (void)hipHostFree(h->h_fl);
    (void)hipHostFree(h->h_sc);
    delete h;
    return hip_fail(e, "solver prepare");
  }
  for (int k = 0; k < h->nrhs; ++k) {
    if (!std::isfinite(h->h_sc[k * SC_COUNT + SC_B2])) {
      (void)hipHostFree(h->h_fl);
      (void)hipHostFree(h->h_sc);
      delete h;
      return fail(WD_EINVAL, "source contains NaN or Inf");
    }
    if (h->h_fl[k * FL_COUNT + FL_CONV]) {
      h->done_rhs[k] = 1;
      h->status[k] = WD_OK;
    }
  }
  *out = h;
  return WD_OK;
}

}  // extern "C"

namespace wd {

bool solver_finished(wd_solver* h) {
  if (h->finished) return true;
  bool any = false;
  for (int k = 0; k < h->nrhs; ++k) any |= !h->done_rhs[k];
  if (!any || h->loops >= h->prm.maxiter) h->finished = true;
  return h->finished;
}

// Launch per_check iterations and the asynchronous copy of their flags;
// returns at once.  An RHS that triggers a reliable update, converges or
// breaks down is paused on the device (its active flag), so the iterations
// after it in the same batch leave it untouched and the result does not
// depend on per_check.
static hipError_t issue_body(wd_solver* h) {
  for (int i = 0; i < h->per_check; ++i) WD_TRY(iteration_body(h));
  return hipSuccess;
}

hipError_t solver_issue(wd_solver* h) {
  hipError_t e = hipSuccess;
  if (h->prm.use_graph && h->s) {
    if (!h->graph_ready) {
      e = hipStreamBeginCapture(h->s, hipStreamCaptureModeRelaxed);
      if (e == hipSuccess) {
        hipError_t eb = issue_body(h);
        e = hipStreamEndCapture(h->s, &h->graph);
        if (eb != hipSuccess) e = eb;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0);
      if (e == hipSuccess) h->graph_ready = true;
    }
    if (e == hipSuccess) e = hipGraphLaunch(h->gexec, h->s);
  } else {
    e = issue_body(h);
  }
  // only the flags come back every iteration; the scalars are read when a
  // breakdown is reported, at a reliable update and at the end
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->h_fl, h->fl, sizeof(int) * FL_COUNT * h->nrhs, hipMemcpyDeviceToHost, h->s);
  return e;
}

// Wait for the issued iterations, account for them, and run the reliable
// update of the RHS that triggered one (CG: then their search-direction
// update).  Iterations are counted on the device (FL_ITERS); a reliable
// update counts as one more (k + l).
wd_status solver_complete(wd_solver* h) {
  hipError_t e = hipStreamSynchronize(h->s);
  if (e != hipSuccess) return hip_fail(e, "solver iteration");
  for (int k = 0; k < h->nrhs; ++k)
    if (!h->done_rhs[k] && h->h_fl[k * FL_COUNT + FL_BREAK]) {
      e = read_flags(h);  // the breakdown note quotes the scalars
      if (e != hipSuccess) return hip_fail(e, "solver iteration");
      break;
    }
  {
    h->loops += h->per_check;
    bool any_ru = false;
    for (int k = 0; k < h->nrhs; ++k) {
      if (h->done_rhs[k]) continue;
      h->iters[k] = h->h_fl[k * FL_COUNT + FL_ITERS] + h->rus[k];
      if (h->h_fl[k * FL_COUNT + FL_BREAK]) {
        h->done_rhs[k] = 1;
        h->status[k] = WD_EBREAKDOWN;
        note_breakdown(h, k);
        continue;
      }
      if (h->h_fl[k * FL_COUNT + FL_RU]) any_ru = true;
    }
    if (any_ru) {
      e = reliable_update(h);
      if (e == hipSuccess) e = read_flags(h);
      if (e != hipSuccess) return hip_fail(e, "reliable update");
      ++h->loops;
      for (int k = 0; k < h->nrhs; ++k) {
        if (h->done_rhs[k] || !h->h_fl[k * FL_COUNT + FL_RU]) continue;
        ++h->rus[k];
        h->iters[k] = h->h_fl[k * FL_COUNT + FL_ITERS] + h->rus[k];
        if (h->h_fl[k * FL_COUNT + FL_CONV]) {
          h->done_rhs[k] = 1;
          h->status[k] = WD_OK;
        } else if (h->h_fl[k * FL_COUNT + FL_BREAK]) {
          h->done_rhs[k] = 1;
          h->status[k] = WD_EBREAKDOWN;
          note_breakdown(h, k);
        }
      }
      if (h->kind == WD_SOLVER_CG) {
        // p = r^ + beta p for the updated RHS that iterate on (rumask)
        e = blas_cg_p(h->geom, h->prm.inner, h->p, h->rh, h->sc, h->rumask, h->s);
        if (e != hipSuccess) return hip_fail(e, "cg p update");
      }
    }
  }
  solver_finished(h);
  return WD_OK;
}

}  // namespace wd

extern "C" {

wd_status wd_solver_step(wd_solver* h, int32_t n_iters, int32_t* done) {
  set_error("");
  if (!h) return fail(WD_EINVAL, "solver handle is NULL");
  if (n_iters < 1) return fail(WD_EINVAL, "n_iters must be >= 1");
  for (int it = 0; it < n_iters && !solver_finished(h); ++it) {
    hipError_t e = solver_issue(h);
    if (e != hipSuccess) return hip_fail(e, "solver iteration");
    wd_status st = solver_complete(h);
    if (st) return st;
  }
  if (done) *done = solver_finished(h) ? 1 : 0;
  return WD_OK;
}

wd_status wd_solver_residuals(wd_solver* h, double* out) {
  set_error("");
  if (!h || !out) return fail(WD_EINVAL, "solver handle or out is NULL");
  hipError_t e = read_flags(h);
  if (e != hipSuccess) return hip_fail(e, "wd_solver_residuals");
  for (int k = 0; k < h->nrhs; ++k) {
    out[3 * k] = h->h_sc[k * SC_COUNT + SC_R2];
    out[3 * k + 1] = h->h_sc[k * SC_COUNT + SC_RTRUE2];
    out[3 * k + 2] = h->h_sc[k * SC_COUNT + SC_B2];
  }
  return WD_OK;
}

wd_status wd_solver_end(wd_solver* h, wd_solve_info* info) {
  set_error("");
  if (!h) return fail(WD_EINVAL, "solver handle is NULL");
  hipError_t e = reconstruct(h);
  if (e == hipSuccess) e = read_flags(h);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - h->t0).count();
  wd_status result = WD_OK;
  if (e != hipSuccess) result = hip_fail(e, "solver end");
  for (int k = 0; k < h->nrhs && result != WD_EDEVICE; ++k) {
    const double* s = h->h_sc + k * SC_COUNT;
    const double rel = (s[SC_B2] > 0) ? std::sqrt(s[SC_RTRUE2] / s[SC_B2]) : 0.0;
    if (info) {
      info[k].iters = h->iters[k];
      info[k].reliable_updates = h->rus[k];
      info[k].converged = (h->status[k] == WD_OK) ? 1 : 0;
      info[k].status = h->status[k];
      info[k].true_rel_resid = rel;
      info[k].seconds = secs;
      const double fl = (h->iters[k] - h->rus[k]) * flops_per_iter(h->kind) +
                        h->rus[k] * flops_per_update(h->kind);
      info[k].gflops = secs > 0 ? fl * h->geom.Vh / secs * 1e-9 : 0.0;
    }
    if (h->status[k] == WD_EBREAKDOWN) result = WD_EBREAKDOWN;
    else if (h->status[k] != WD_OK && result == WD_OK) result = WD_NOT_CONVERGED;
  }
  if (h->graph_ready) {
    (void)hipGraphExecDestroy(h->gexec);
    (void)hipGraphDestroy(h->graph);
  }
  (void)hipHostFree(h->h_fl);
  (void)hipHostFree(h->h_sc);
  const std::string note = h->note;
  delete h;
  if (result == WD_NOT_CONVERGED) set_error("maxiter reached before the target residual");
  if (result == WD_EBREAKDOWN) set_error("Krylov recurrence broke down:" + note);
  return result;
}

static wd_status solve(int kind, const wd_gauge* g, double kappa, double* x, const double* b,
                       const wd_solve_params* prm, wd_solve_info* info, void* ws, size_t ws_bytes,
                       void* stream) {
  wd_solver* h = nullptr;
  wd_status st = wd_solver_begin(kind, g, kappa, x, b, prm, ws, ws_bytes, stream, &h);
  if (st) return st;
  int done = 0;
  while (!done) {
    st = wd_solver_step(h, 1 << 20, &done);
    if (st) {
      std::string msg = wd_last_error();
      wd_solver_end(h, nullptr);
      return fail(st, msg);
    }
  }
  return wd_solver_end(h, info);
}

wd_status bicgstab_solve(const wd_gauge* g, double kappa, double* x, const double* b,
                         const wd_solve_params* params, wd_solve_info* info, void* workspace,
                         size_t ws_bytes, void* stream) {
  return solve(WD_SOLVER_BICGSTAB, g, kappa, x, b, params, info, workspace, ws_bytes, stream);
}

wd_status cg_solve(const wd_gauge* g, double kappa, double* x, const double* b,
                   const wd_solve_params* params, wd_solve_info* info, void* workspace,
                   size_t ws_bytes, void* stream) {
  return solve(WD_SOLVER_CG, g, kappa, x, b, params, info, workspace, ws_bytes, stream);
}

}  // extern "C"
