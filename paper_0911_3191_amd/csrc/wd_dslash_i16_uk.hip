// Dslash kernels of one storage format (SI16) on UKQCD-basis fields, the
// basis the solvers work in; see wd_dslash_impl.h.
#include "wd_dslash_impl.h"

namespace wd {

void launch_dslash_i16_uk(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s) {
  launch_cfg<SI16, kBasisUK>(g, d, c, s);
}

}  // namespace wd
