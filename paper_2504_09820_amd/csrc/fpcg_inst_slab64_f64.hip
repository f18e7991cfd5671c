// Slab-kernel instantiations for K = 64 with FP64 operands.
#include "fpcg_registry.hpp"

namespace fpcg {

void register_slab64_f64(std::vector<KernelEntry>& v) {
    FPCG_SLAB_IO(64, F64, 0);
    FPCG_SLAB_IO(64, F64, 4);
}

}  // namespace fpcg
