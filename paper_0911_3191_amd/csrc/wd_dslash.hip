// Dslash entry points: dispatch to the per-format launchers, tuned launch
// shapes, partial-record counts (kernels: wd_dslash_impl.h).
#include "wd_dslash_impl.h"

namespace wd {

void launch_dslash_fp64(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s);
void launch_dslash_fp32(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s);
void launch_dslash_i16(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s);
void launch_dslash_f16(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s);
void launch_dslash_fp64_uk(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s);
void launch_dslash_fp32_uk(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s);
void launch_dslash_i16_uk(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s);
void launch_dslash_f16_uk(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s);

void launch_dslash_cfg(const wd_gauge* g, wd_prec prec, const DslashArgs& d, const LaunchCfg& c,
                       hipStream_t s) {
  const bool uk = d.basis == kBasisUK;
  switch (prec) {
    case WD_FP64: uk ? launch_dslash_fp64_uk(g, d, c, s) : launch_dslash_fp64(g, d, c, s); break;
    case WD_FP32: uk ? launch_dslash_fp32_uk(g, d, c, s) : launch_dslash_fp32(g, d, c, s); break;
    case WD_HALF_I16: uk ? launch_dslash_i16_uk(g, d, c, s) : launch_dslash_i16(g, d, c, s); break;
    default: uk ? launch_dslash_f16_uk(g, d, c, s) : launch_dslash_f16(g, d, c, s); break;
  }
}

hipError_t launch_dslash_ex(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s) {
  if (prec < WD_FP64 || prec > WD_HALF_F16) return hipErrorInvalidValue;
  if (d.basis != kBasisDR && d.basis != kBasisUK) return hipErrorInvalidValue;
  if (d.basis == kBasisDR && d.xpay && d.dot != DOT_NONE) return hipErrorInvalidValue;
  if (d.rhs_map && (d.n_map < 1 || d.n_map > d.out.nrhs)) return hipErrorInvalidValue;
  if (d.dot == DOT_RES && (prec != WD_FP64 || !d.xpay || !d.y || d.dagger)) return hipErrorInvalidValue;
  if (d.dot == DOT_RES_ENC &&
      (prec != WD_FP64 || !d.xpay || !d.y || d.dagger || d.basis != kBasisUK || !d.enc_rh || !d.enc_xh ||
       !d.enc_rt || d.enc_prec < WD_FP32 || d.enc_prec > WD_HALF_F16))
    return hipErrorInvalidValue;
  if (d.dot == DOT_ENC && (prec != WD_FP64 || !d.xpay || !d.dagger || d.basis != kBasisUK || !d.enc_rh ||
                           !d.enc_xh || d.enc_prec < WD_FP32 || d.enc_prec > WD_HALF_F16))
    return hipErrorInvalidValue;
  LaunchCfg c = tuned_dslash_config(g, prec, d, s);
  // A fused dot sums each workgroup's sites into one partial record; with one
  // sub-slab and 256-thread workgroups those site sets are fixed whatever the
  // other fields are, so the reduction -- and the solver -- give the same bits
  // for every tuned shape.
  if (d.xpay && d.dot != DOT_NONE) {
    c.nsub = 1;
    c.block = 256;
  }
  launch_dslash_cfg(g, prec, d, c, s);
  return hipGetLastError();
}

hipError_t launch_dslash(const wd_gauge* g, wd_prec prec, Field out, Field in, int out_parity,
                         int dagger, const Field* xpay_src, double a, hipStream_t s, int basis) {
  DslashArgs d;
  d.out = out;
  d.in = in;
  d.out_parity = out_parity;
  d.dagger = dagger;
  d.xpay = xpay_src;
  d.a = a;
  d.basis = basis;
  return launch_dslash_ex(g, prec, d, s);
}

int dslash_partial_blocks(const Geom& geo, int nrhs, const LaunchCfg& c) {
  const DslashGeom g = make_dgeom(geo, nrhs, c);
  return (g.slab ? 8 : 1) * g.site_blocks;
}

}  // namespace wd
