// Slab-kernel instantiations for K = 64 with reduced and FP32 operands
// (four waves per channel, A held in registers).
#include "fpcg_registry.hpp"

namespace fpcg {

void register_slab64(std::vector<KernelEntry>& v) {
    FPCG_SLAB_IO(64, F16, 0);
    FPCG_SLAB_IO(64, F16, 4);
    FPCG_SLAB_IO(64, BF16, 0);
    FPCG_SLAB_IO(64, BF16, 4);
    FPCG_SLAB_IO(64, F32, 0);
    FPCG_SLAB_IO(64, F32, 4);
    FPCG_SLAB_IO(64, F32, 16);
}

}  // namespace fpcg
