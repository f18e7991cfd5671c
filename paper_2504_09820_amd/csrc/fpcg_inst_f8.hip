// Fused-kernel instantiations for the fp8 e4m3 operand format (the 16x16x32
// fp8 matrix-core shape needs 8 contraction values per lane: padded K >= 32).
#include "fpcg_registry.hpp"

namespace fpcg {

void register_f8(std::vector<KernelEntry>& v) {
    FPCG_ENTRIES_IO(32, F8, 0);
    FPCG_ENTRIES_IO(32, F8, 4);
    FPCG_ENTRIES_IO(32, F8, 8);
    FPCG_ENTRIES_IO(64, F8, 0);
    FPCG_ENTRIES_IO(64, F8, 4);
    FPCG_ENTRIES_IO(64, F8, 8);
}

}  // namespace fpcg
