// Fused-kernel instantiations for the BF16 operand format.
#include "fpcg_registry.hpp"

namespace fpcg {

void register_bf16(std::vector<KernelEntry>& v) {
    FPCG_ENTRIES_IO(16, BF16, 0);
    FPCG_ENTRIES_IO(16, BF16, 4);
    FPCG_ENTRIES_IO(32, BF16, 0);
    FPCG_ENTRIES_IO(32, BF16, 4);
    FPCG_ENTRIES_IO(32, BF16, 8);
    FPCG_ENTRIES_IO(64, BF16, 0);
    FPCG_ENTRIES_IO(64, BF16, 4);
    FPCG_ENTRIES_IO(64, BF16, 8);
}

}  // namespace fpcg
