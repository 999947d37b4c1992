// Internal declarations shared by the host and device translation units of
// libwdslash.so.  Not part of the public ABI (include/wd.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "wd.h"

namespace wd {

// Lattice geometry as the kernels see it.  Every field of one lattice uses the
// same per-chunk site stride `stride` (>= Vh, padded, see field_stride).
struct Geom {
  int L[4];     // Lx, Ly, Lz, Lt
  int Lxh;      // Lx / 2
  int Vh;       // sites per parity
  int tap;      // antiperiodic in t
  int64_t stride;
};

Geom make_geom(const wd_lattice& lat);
int64_t field_stride(int64_t Vh);

// Bytes of one real in each storage precision and the number of 16-byte
// chunks a site's 24 spinor reals occupy.
inline int spinor_chunks(wd_prec p) { return p == WD_FP64 ? 12 : (p == WD_FP32 ? 6 : 3); }
inline bool is_half(wd_prec p) { return p == WD_HALF_I16 || p == WD_HALF_F16; }
// Bytes per stored link: 12 reals (Appendix A.1) or 8 reals (Appendix A.2).
inline int link_bytes(wd_prec p, int recon = 12) {
  const int reals = recon == 8 ? 8 : 12;
  return reals * (p == WD_FP64 ? 8 : (p == WD_FP32 ? 4 : 2));
}

// A parity spinor field: nrhs right-hand sides, chunk arrays of `stride`
// 16-byte elements each, laid out [rhs][chunk][site]; 16-bit formats append
// a binary32 norm array [rhs][site] after all chunks.
struct Field {
  char* ptr;
  int64_t stride;
  int nrhs;
};

size_t spinor_field_bytes(const Geom& g, wd_prec p, int nrhs);
// Bytes of one field of the canonical operators' workspace (rounded up to
// 256 so every field starts aligned); the workspace holds four.
size_t operator_field_slot(const Geom& g, wd_prec prec, int nrhs);

}  // namespace wd

struct wd_gauge {
  wd_lattice lat;
  wd::Geom geom;
  uint32_t mask;
  int recon;      // 12 or 8 reals per link
  int tgauge;     // 1: temporal links are the unit matrix except on the last time slice
  void* link[4];  // per precision: [parity][mu][chunk][site]
};

namespace wd {

// ---- launchers (defined in the .hip files; all asynchronous on `s`) -------------
constexpr int kMaxDotHost = 4;  // doubles per partial record
// DOT_RES (FP64 only): out = y - (xpay + a D in), the residual of a reliable
// update, with |out|^2 partials.  DOT_RES_ENC (FP64, UKQCD basis): the same
// residual r is not stored in FP64 but re-encoded straight into the inner
// solver's fields: enc_rh = enc(r), enc_xh = 0 (with enc_set_rt also the new
// shadow residual enc_rt = enc(r), as defect correction restarts from it),
// partials |r|^2, |enc(r)|^2, <enc_rt, enc(r)> (the last two on the stored
// values).  DOT_ENC (FP64 adjoint, UKQCD basis): out = xpay + a D^dag in is
// not stored in FP64 but encoded straight into enc_rh, enc_xh = 0, partial
// |enc_rh|^2 on the stored value (CG's reliable update: r^ = enc(M_hat^dag r)).
enum DotMode { DOT_NONE = 0, DOT_YO = 1, DOT_OX = 2, DOT_OO = 3, DOT_RES = 4, DOT_RES_ENC = 5, DOT_ENC = 6 };

// Full argument set of one dslash launch.  out = D in, or, with xpay set,
// out = *xpay + a * D in; with xpay and dot set, per-block FP64 partials of
// the dot products named by DotMode go to partials[rhs][block][4].  RHS whose
// active flag is 0 are skipped.
// Spin bases of spinor fields (Appendix B): the caller's fields are in the
// DeGrand-Rossi basis, the solvers rotate theirs into the UKQCD basis.
constexpr int kBasisDR = 0, kBasisUK = 1;

struct DslashArgs {
  Field out{}, in{};
  int out_parity = 0, dagger = 0;
  const Field* xpay = nullptr;
  double a = 0.0;
  int dot = DOT_NONE;
  const Field* y = nullptr;
  double* partials = nullptr;
  const int* active = nullptr;  // device mask [nrhs]: RHS with 0 are skipped
  // Device list of n_map RHS indices (distinct, < out.nrhs): only those are
  // processed, packed into as few RHS groups as they fill (replaces `active`).
  const int* rhs_map = nullptr;
  int n_map = 0;
  int basis = kBasisDR;  // spin basis of the fields (fused dots: UKQCD only)
  // DOT_RES_ENC: the inner precision and its residual, zeroed solution and
  // shadow residual fields
  wd_prec enc_prec = WD_FP32;
  const Field* enc_rh = nullptr;
  const Field* enc_xh = nullptr;
  const Field* enc_rt = nullptr;
  int enc_set_rt = 0;
  // 1: never run the autotuner for this launch (a tuned shape already cached
  // is used, else the default); for callers that must not create events
  int no_tune = 0;
};
hipError_t launch_dslash_ex(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s);

// Launch shape of the dslash: right-hand sides per thread and threads per
// workgroup.  The workgroup size is fixed at 256 so that fused dot products
// reduce in the same order whatever the batch; only nr is tuned.
struct LaunchCfg {
  int nr;
  int block;
  int gslow = 0;    // RHS group slowest in an XCD's sweep (else fastest)
  int nsub = 1;     // y-sub-slabs an XCD sweeps one after the other
  int link_nt = 0;  // link loads marked streaming
  int out_nt = 0;   // output stores marked streaming
  int wgs = 0;      // cap on workgroups per CU (0: registers decide)
  int lds = 0;      // 16-bit formats: stage x/y neighbours in LDS
  int rloop = 0;    // binary16, 12-real links: one thread per site loops over every RHS
};
void launch_dslash_cfg(const wd_gauge* g, wd_prec prec, const DslashArgs& d, const LaunchCfg& c,
                       hipStream_t s);
// Partial records per RHS written by a dslash launch with a fused dot.
int dslash_partial_blocks(const Geom& geo, int nrhs, const LaunchCfg& c);
// Autotuner (wd_tune.cpp): the configuration to use for this launch; times
// the candidates, in the launch's own form and on its own fields, on first
// use of (lattice, precision, RHS count, link format and basis, form) unless
// the stream is being captured.
LaunchCfg tuned_dslash_config(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s);
// Tunes the key of launch d now (the launch itself is not made).
void tune_dslash(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s);

// out_p = D_{p,1-p} in (dagger: adjoint).  When xpay_src is non-null:
// out = xpay_src + a * D in (xpay_src has parity p, same precision).
hipError_t launch_dslash(const wd_gauge* g, wd_prec prec, Field out, Field in, int out_parity,
                         int dagger, const Field* xpay_src, double a, hipStream_t s,
                         int basis = kBasisDR);

hipError_t launch_gauge_encode(const wd_gauge* g, const double* U, hipStream_t s);
// 8-real links, temporal gauge (wd_gauge.hip)
hipError_t launch_gauge_encode8(const wd_gauge* g, const double* U, hipStream_t s);
hipError_t launch_temporal_check(const Geom& geo, const double* U, unsigned long long* dev, hipStream_t s);
hipError_t launch_gauge_fix_temporal(const Geom& geo, const double* U, double* Uo, double* g, hipStream_t s);
hipError_t launch_gauge_rotate(const Geom& geo, const double* g, const double* in, double* out, int nrhs,
                               int adjoint, hipStream_t s);

// canonical parity spinors [nrhs][Vh][24] (DeGrand-Rossi basis) <-> field
// (spin basis `basis`)
hipError_t launch_spinor_encode(const Geom& g, wd_prec p, Field f, const double* canon,
                                hipStream_t s, int basis = kBasisDR);
hipError_t launch_spinor_decode(const Geom& g, wd_prec p, double* canon, Field f,
                                hipStream_t s, int basis = kBasisDR);
// full_parity = p: the canonical array is a full lattice [nrhs][V][24] and the
// field holds (or provides) its parity-p sites; full_parity < 0: parity array.
// scale = 1 / 2: the solver's unit-source scaling, values divided / multiplied
// by the per-RHS |b| held in the solver scalars sc (see SC_BNORM).
hipError_t launch_spinor_encode_map(const Geom& g, wd_prec p, Field f, const double* canon,
                                    int full_parity, hipStream_t s, int basis = kBasisDR,
                                    const double* sc = nullptr, int scale = 0);
hipError_t launch_spinor_decode_map(const Geom& g, wd_prec p, double* canon, Field f,
                                    int full_parity, hipStream_t s, int basis = kBasisDR,
                                    const double* sc = nullptr, int scale = 0);
// Both parities of a full-lattice canonical array in one pass (FP64 fields):
// even sites to / from fe, odd sites to / from fo; scale as above.
hipError_t launch_spinor_encode_both(const Geom& g, Field fe, Field fo, const double* canon, hipStream_t s,
                                     int basis, const double* sc = nullptr, int scale = 0);
hipError_t launch_spinor_decode_both(const Geom& g, double* canon, Field fe, Field fo, hipStream_t s,
                                     int basis, const double* sc = nullptr, int scale = 0);

// ---- solver state on the device --------------------------------------------------
// Per-RHS FP64 scalars (complex ones take two slots: re, im).
enum ScalarSlot {
  SC_RHO = 0,      // rho = <r~, r^> (BiCGstab, complex) or |r^|^2 (CG)
  SC_RHOP = 2,     // previous rho
  SC_ALPHA = 4,    // alpha (complex for BiCGstab)
  SC_OMEGA = 6,    // omega (BiCGstab)
  SC_R2 = 8,       // |r^|^2 of the iterated residual
  SC_RTRUE2 = 9,   // |b_hat - M_hat x|^2 at the last reliable update (FP64)
  SC_MMAX = 10,    // max |r^| since the last reliable update (Algorithm 2's M)
  SC_B2 = 11,      // |b|^2 of the full-lattice source
  SC_TOLN = 12,    // CG: target on the normal-equation residual
  SC_BETA = 13,    // CG: beta
  SC_BNORM = 14,   // |b| of the caller's source (the solve runs on b / |b|)
  SC_COUNT = 16
};
// FL_ITERS counts the inner iterations an RHS has started, on the device, so
// that several iterations can run between two reads of the flags by the host.
enum FlagSlot { FL_RU = 0, FL_BREAK = 1, FL_CONV = 2, FL_ITERS = 3, FL_COUNT = 4 };
enum FinStage {
  FIN_B2, FIN_TRUE, FIN_RHO, FIN_BICG_INIT, FIN_BICG_ALPHA, FIN_BICG_OMEGA,
  FIN_BICG_ITER, FIN_CG_INIT, FIN_CG_ALPHA, FIN_CG_ITER, FIN_CG_RHO,
  FIN_TRUE_RHO,  // FIN_TRUE on v[0], then FIN_RHO on v[1..3] where iteration goes on
  FIN_TRUE_INIT  // FIN_TRUE on v[0], then FIN_BICG_INIT on v[1..3] where iteration goes on
};

hipError_t blas_bicg_p(const Geom& g, wd_prec pr, Field p, Field r, Field v, const double* sc,
                       const int* mask, hipStream_t s);
hipError_t blas_bicg_s(const Geom& g, wd_prec pr, Field r, Field v, const double* sc,
                       const int* mask, hipStream_t s);
hipError_t blas_bicg_xr(const Geom& g, wd_prec pr, Field x, Field r, Field p, Field t, Field rt,
                        const double* sc, const int* mask, double* partials, hipStream_t s);
hipError_t blas_cg_xr(const Geom& g, wd_prec pr, Field x, Field r, Field p, Field q,
                      const double* sc, const int* mask, double* partials, hipStream_t s);
hipError_t blas_cg_p(const Geom& g, wd_prec pr, Field p, Field r, const double* sc,
                     const int* mask, hipStream_t s);
hipError_t blas_convert(const Geom& g, wd_prec dst_prec, Field dst, wd_prec src_prec, Field src,
                        const int* mask, hipStream_t s);
hipError_t blas_zero(const Geom& g, wd_prec pr, Field f, const int* mask, hipStream_t s);
hipError_t blas_norm2(const Geom& g, wd_prec pr, Field f, const int* mask, double* partials,
                      hipStream_t s);
hipError_t blas_accum(const Geom& g, wd_prec pr, Field x64, Field xh, const int* mask, hipStream_t s);
// partials: |b|^2 of a canonical full-lattice FP64 array [nrhs][2 Vh][24], the
// record count per RHS of the BLAS-1 kernels.
hipError_t blas_canon_norm2(const Geom& g, const double* canon, int nrhs, double* partials, hipStream_t s);
// rh <- enc(r64), xh <- 0; partials |rh|^2 and, with rt, <rt, rh>; set_rt
// writes rt <- enc(r64) first (the same bits as rh).
hipError_t blas_reencode(const Geom& g, wd_prec pr, Field rh, Field xh, Field r64, const Field* rt,
                         const int* mask, double* partials, hipStream_t s, bool set_rt = false);
// restart = 1 (defect correction): the update trigger compares |r^| with the
// residual the inner solve started from, and CG restarts with beta = 0.
hipError_t solver_finalize(int stage, int nrhs, int nb, const double* partials, double* sc, int* fl,
                           int* active, int* rumask, const int* mask, double delta, double tol,
                           int restart, hipStream_t s);
hipError_t solver_cg_tighten(int nrhs, double* sc, const int* fl, const int* mask, double tol,
                             hipStream_t s);
hipError_t solver_init_flags(int nrhs, int* fl, int* active, int* rumask, hipStream_t s);

// ---- two-phase stepping (wd_solver.cpp), used by the serving scheduler ---------------
bool solver_finished(wd_solver* h);
hipError_t solver_issue(wd_solver* h);   // launch one iteration, returns at once
wd_status solver_complete(wd_solver* h); // wait for it, reliable update if triggered

// Canonical FP64 parity spinors in, encoded fields of `prec` in the
// workspace `ws` (four fields of `slot` bytes), canonical out: op 0 is the
// hopping term D_{p,1-p}, op 1 M_hat (adjoint with dagger), op 2
// M_hat^dagger M_hat.  Asynchronous on s.
// no_tune: the dslash launches never run the autotuner.
hipError_t canon_operator(const wd_gauge* g, int op, double kappa, double* out, const double* in,
                          int out_parity, int dagger, wd_prec prec, int nrhs, char* ws, size_t slot,
                          hipStream_t s, bool no_tune = false);

// ---- error reporting ------------------------------------------------------------
void set_error(const std::string& msg);
wd_status fail(wd_status code, const std::string& msg);

}  // namespace wd
