// Fused-kernel instantiations for the F64 operand format.
#include "fpcg_registry.hpp"

namespace fpcg {

void register_f64(std::vector<KernelEntry>& v) {
    FPCG_ENTRIES_IO(16, F64, 0);
    FPCG_ENTRIES_IO(16, F64, 4);
    FPCG_ENTRIES_IO(32, F64, 0);
    FPCG_ENTRIES_IO(32, F64, 4);
    FPCG_ENTRIES_IO(32, F64, 8);
    FPCG_ENTRIES_IO(64, F64, 0);
    FPCG_ENTRIES_IO(64, F64, 4);
    FPCG_ENTRIES_IO(64, F64, 8);
}

}  // namespace fpcg
