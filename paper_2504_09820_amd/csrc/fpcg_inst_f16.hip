// Fused-kernel instantiations for the F16 operand format.
#include "fpcg_registry.hpp"

namespace fpcg {

void register_f16(std::vector<KernelEntry>& v) {
    FPCG_ENTRIES_IO(16, F16, 0);
    FPCG_ENTRIES_IO(16, F16, 4);
    FPCG_ENTRIES_IO(32, F16, 0);
    FPCG_ENTRIES_IO(32, F16, 4);
    FPCG_ENTRIES_IO(32, F16, 8);
    FPCG_ENTRIES_IO(64, F16, 0);
    FPCG_ENTRIES_IO(64, F16, 4);
    FPCG_ENTRIES_IO(64, F16, 8);
}

}  // namespace fpcg
