// Fused-kernel instantiations for K = 64 with fp16 / bf16 operands and more
// than one wave per channel (four waves: L <= 4; two waves: L <= 8).
#include "fpcg_registry.hpp"

namespace fpcg {

void register_k64w_f16(std::vector<KernelEntry>& v) {
    FPCG_ENTRIES_IO_NW(64, F16, 0, 4);
    FPCG_ENTRIES_IO_NW(64, F16, 4, 4);
    FPCG_ENTRIES_IO_NW(64, F16, 8, 2);
    FPCG_ENTRIES_IO_NW(64, BF16, 0, 4);
    FPCG_ENTRIES_IO_NW(64, BF16, 4, 4);
    FPCG_ENTRIES_IO_NW(64, BF16, 8, 2);
}

}  // namespace fpcg
