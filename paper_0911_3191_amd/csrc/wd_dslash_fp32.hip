// Dslash kernels of one storage format (SF32) on DeGrand-Rossi-basis fields;
// see wd_dslash_impl.h.
#include "wd_dslash_impl.h"

namespace wd {

void launch_dslash_fp32(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s) {
  launch_cfg<SF32, kBasisDR>(g, d, c, s);
}

}  // namespace wd
