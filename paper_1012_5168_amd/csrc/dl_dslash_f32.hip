// dl_dslash_f32.hip -- hopping kernels with float storage.
#include "dl_dslash_inst.hpp"

namespace dl {
template void launch_dslash_t<float>(const DslashCall *c, int nseg, int kind, int nr, int bs,
                                        int persistent, hipStream_t s);
}  // namespace dl
