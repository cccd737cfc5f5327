// dl_dslash_bf16.hip -- hopping kernels with __hip_bfloat16 storage.
#include "dl_dslash_inst.hpp"

namespace dl {
template void launch_dslash_t<__hip_bfloat16>(const DslashCall *c, int nseg, int kind, int nr, int bs,
                                        int persistent, hipStream_t s);
}  // namespace dl
