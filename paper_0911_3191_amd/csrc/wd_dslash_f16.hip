// Dslash kernels of one storage format (SF16) on DeGrand-Rossi-basis fields;
// see wd_dslash_impl.h.
#include "wd_dslash_impl.h"

namespace wd {

void launch_dslash_f16(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s) {
  launch_cfg<SF16, kBasisDR>(g, d, c, s);
}

}  // namespace wd
