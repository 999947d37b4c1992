// Dslash kernels of one storage format (SI16); see wd_dslash_impl.h.
#include "wd_dslash_impl.h"

namespace wd {

void launch_dslash_i16(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s) {
  launch_cfg<SI16>(g, d, c, s);
}

}  // namespace wd
