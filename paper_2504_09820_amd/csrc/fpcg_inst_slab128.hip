// Slab-kernel instantiations for K = 128 (eight waves per channel) with FP64
// and FP32 operands: the u_W matrix does not fit LDS beside the rest, so only
// the register-resident layout holds it.  FP32, fp16 and bf16 also with
// L = 16 in the symmetric form (with or without the FP64 refresh).
#include "fpcg_registry.hpp"

namespace fpcg {

void register_slab128(std::vector<KernelEntry>& v) {
    FPCG_SLAB_IO(128, F64, 0);
    FPCG_SLAB_IO(128, F32, 0);
    FPCG_SLAB_IO(128, F32, 16);
    FPCG_SLAB_IO(128, F16, 16);
    FPCG_SLAB_IO(128, BF16, 16);
}

}  // namespace fpcg
