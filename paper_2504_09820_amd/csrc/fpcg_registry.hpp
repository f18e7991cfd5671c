// Table of compiled fused-kernel variants (one per padded K, waves per
// channel, operand format, Jacobi block size and I/O element type).
#pragma once

#include <hip/hip_runtime.h>
#include <vector>

#include "fpcg_fused.hpp"

namespace fpcg {

struct KernelEntry {
    int KP, NW, FMT, LB, io_c64;
    size_t lds;
    const void* fn;
    void (*launch)(const FusedParams&, dim3, hipStream_t);
};

void register_f64(std::vector<KernelEntry>& v);
void register_f32(std::vector<KernelEntry>& v);
void register_bf16(std::vector<KernelEntry>& v);
void register_f16(std::vector<KernelEntry>& v);
void register_f8(std::vector<KernelEntry>& v);

// waves per channel for a padded K
constexpr int waves_for(int KP) { return KP >= 64 ? 2 : 1; }

#define FPCG_ENTRY(KP_, FMT_, LB_, IOT_)                                                          \
    do {                                                                                          \
        constexpr int NW_ = waves_for(KP_);                                                       \
        using C_ = Cfg<KP_, NW_, FMT_, LB_>;                                                      \
        KernelEntry e;                                                                            \
        e.KP = KP_; e.NW = NW_; e.FMT = FMT_; e.LB = LB_;                                         \
        e.io_c64 = sizeof(IOT_) == 4 ? 1 : 0;                                                     \
        e.lds = C_::lds_bytes;                                                                    \
        e.fn = reinterpret_cast<const void*>(&fused_kernel<KP_, NW_, FMT_, LB_, IOT_>);           \
        e.launch = [](const FusedParams& p, dim3 grid, hipStream_t s) {                           \
            hipLaunchKernelGGL((fused_kernel<KP_, NW_, FMT_, LB_, IOT_>), grid, dim3(64 * NW_),   \
                               C_::lds_bytes, s, p);                                              \
        };                                                                                        \
        v.push_back(e);                                                                           \
    } while (0)

#define FPCG_ENTRIES_IO(KP_, FMT_, LB_) \
    FPCG_ENTRY(KP_, FMT_, LB_, float);  \
    FPCG_ENTRY(KP_, FMT_, LB_, double)

}  // namespace fpcg
