// Fused-kernel instantiations for K up to 128 with fp16 / bf16 operands (two
// waves per channel, A kept in the operand format).
#include "fpcg_registry.hpp"

namespace fpcg {

void register_k128_f16(std::vector<KernelEntry>& v) {
    FPCG_ENTRIES_IO(128, F16, 0);
    FPCG_ENTRIES_IO(128, F16, 16);
    FPCG_ENTRIES_IO(128, BF16, 0);
    FPCG_ENTRIES_IO(128, BF16, 16);
}

}  // namespace fpcg
