// dl_dslash_f16.hip -- hopping kernels with __half storage.
#include "dl_dslash_inst.hpp"

namespace dl {
template void launch_dslash_t<__half>(const DslashCall *c, int nseg, int kind, int nr, int bs,
                                        int persistent, hipStream_t s);
}  // namespace dl
