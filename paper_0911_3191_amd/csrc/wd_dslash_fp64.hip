// Dslash kernels of one storage format (SF64) on DeGrand-Rossi-basis fields;
// see wd_dslash_impl.h.
#include "wd_dslash_impl.h"

namespace wd {

void launch_dslash_fp64(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s) {
  launch_cfg<SF64, kBasisDR>(g, d, c, s);
}

}  // namespace wd
