// Slab-kernel instantiations for K = 64 with reduced and FP32 operands
// (four waves per channel, A held in registers); L = 8 and 16 in the
// symmetric form only.
#include "fpcg_registry.hpp"

namespace fpcg {

void register_slab64(std::vector<KernelEntry>& v) {
    FPCG_SLAB_IO(64, F16, 0);
    FPCG_SLAB_IO(64, F16, 4);
    FPCG_SLAB_IO(64, F16, 8);
    FPCG_SLAB_IO(64, BF16, 0);
    FPCG_SLAB_IO(64, BF16, 4);
    FPCG_SLAB_IO(64, BF16, 8);
    FPCG_SLAB_IO(64, F32, 0);
    FPCG_SLAB_IO(64, F32, 4);
    FPCG_SLAB_IO(64, F32, 8);
    FPCG_SLAB_IO(64, F32, 16);
}

}  // namespace fpcg
