// Fused-kernel instantiations for K up to 128 with fp8 operands (two waves
// per channel, A kept in the operand format).
#include "fpcg_registry.hpp"

namespace fpcg {

void register_k128_f8(std::vector<KernelEntry>& v) {
    FPCG_ENTRIES_IO(128, F8, 0);
    FPCG_ENTRIES_IO(128, F8, 8);
    FPCG_ENTRIES_IO(128, F8, 16);
}

}  // namespace fpcg
