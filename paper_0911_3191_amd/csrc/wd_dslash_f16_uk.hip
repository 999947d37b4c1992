// Dslash kernels of one storage format (SF16) on UKQCD-basis fields, the
// basis the solvers work in; see wd_dslash_impl.h.
#include "wd_dslash_impl.h"

namespace wd {

void launch_dslash_f16_uk(const wd_gauge* g, const DslashArgs& d, const LaunchCfg& c, hipStream_t s) {
  launch_cfg<SF16, kBasisUK>(g, d, c, s);
}

}  // namespace wd
