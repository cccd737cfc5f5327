// dl_dslash_f64.hip -- hopping kernels with double storage.
#include "dl_dslash_inst.hpp"

namespace dl {
template void launch_dslash_t<double>(const DslashCall *c, int nseg, int kind, int nr, int bs,
                                        int persistent, hipStream_t s);
}  // namespace dl
