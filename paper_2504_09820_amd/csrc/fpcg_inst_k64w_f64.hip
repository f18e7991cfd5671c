// Fused-kernel instantiations for K = 64 with FP64 and FP32 operands and four
// waves per channel (the operand copy of A held in registers).
#include "fpcg_registry.hpp"

namespace fpcg {

void register_k64w_f64(std::vector<KernelEntry>& v) {
    FPCG_ENTRIES_IO_NW(64, F64, 0, 4);
    FPCG_ENTRIES_IO_NW(64, F64, 4, 4);
    FPCG_ENTRIES_IO_NW(64, F32, 0, 4);
    FPCG_ENTRIES_IO_NW(64, F32, 4, 4);
}

}  // namespace fpcg
