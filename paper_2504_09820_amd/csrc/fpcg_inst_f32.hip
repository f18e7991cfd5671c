// Fused-kernel instantiations for the F32 operand format.
#include "fpcg_registry.hpp"

namespace fpcg {

void register_f32(std::vector<KernelEntry>& v) {
    FPCG_ENTRIES_IO(16, F32, 0);
    FPCG_ENTRIES_IO(16, F32, 4);
    FPCG_ENTRIES_IO(32, F32, 0);
    FPCG_ENTRIES_IO(32, F32, 4);
    FPCG_ENTRIES_IO(32, F32, 8);
    FPCG_ENTRIES_IO(64, F32, 0);
    FPCG_ENTRIES_IO(64, F32, 4);
    FPCG_ENTRIES_IO(64, F32, 8);
}

}  // namespace fpcg
