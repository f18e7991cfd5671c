// Table of compiled fused-kernel variants (one per padded K, waves per
// channel, operand format, Jacobi block size and I/O element type).
#pragma once

#include <hip/hip_runtime.h>
#include <vector>

#include "fpcg_fused.hpp"

namespace fpcg {

struct KernelEntry {
    int KP, NW, FMT, LB, io_c64;
    size_t lds, lds_refine;     // dynamic LDS without / with FP64 refinement
    const void* fn;
    void (*launch)(const FusedParams&, dim3, size_t, hipStream_t);
};

void register_f64(std::vector<KernelEntry>& v);
void register_f32(std::vector<KernelEntry>& v);
void register_bf16(std::vector<KernelEntry>& v);
void register_f16(std::vector<KernelEntry>& v);
void register_f8(std::vector<KernelEntry>& v);

// waves per channel for a padded K and operand format: one wave holds the
// whole iterate (K/4 complex entries per lane) except where the FP64 vectors
// would not fit the register file
constexpr int waves_for(int KP, int FMT) { return (FMT == F64 && KP >= 64) ? 2 : 1; }

#define FPCG_ENTRY(KP_, FMT_, LB_, IOT_)                                                          \
    do {                                                                                          \
        constexpr int NW_ = waves_for(KP_, FMT_);                                                       \
        using C_ = Cfg<KP_, NW_, FMT_, LB_>;                                                      \
        KernelEntry e;                                                                            \
        e.KP = KP_; e.NW = NW_; e.FMT = FMT_; e.LB = LB_;                                         \
        e.io_c64 = sizeof(IOT_) == 4 ? 1 : 0;                                                     \
        e.lds = C_::lds_bytes;                                                                    \
        e.lds_refine = C_::lds_bytes_refine;                                                      \
        e.fn = reinterpret_cast<const void*>(&fused_kernel<KP_, NW_, FMT_, LB_, IOT_>);           \
        e.launch = [](const FusedParams& p, dim3 grid, size_t lds, hipStream_t s) {               \
            hipLaunchKernelGGL((fused_kernel<KP_, NW_, FMT_, LB_, IOT_>), grid, dim3(64 * NW_),   \
                               lds, s, p);                                                        \
        };                                                                                        \
        v.push_back(e);                                                                           \
    } while (0)

#define FPCG_ENTRIES_IO(KP_, FMT_, LB_) \
    FPCG_ENTRY(KP_, FMT_, LB_, float);  \
    FPCG_ENTRY(KP_, FMT_, LB_, double)

}  // namespace fpcg
