// Table of compiled fused-kernel variants (one per padded K, waves per
// channel, operand format, Jacobi block size and I/O element type).
#pragma once

#include <hip/hip_runtime.h>
#include <vector>

#include "fpcg_fused.hpp"
#include "fpcg_slab.hpp"

namespace fpcg {

struct KernelEntry {
    int KP, NW, FMT, LB, io_c64;                 // NW: waves per channel
    int kind = 0;                                // 0: fused_kernel; 1: slab_kernel (fn[sp][1]: the refresh build)
    int arow = 0;               // A kept only in the operand format (no u_W Gram in LDS)
    size_t (*lds)(bool split, bool refine, int refresh_every);   // dynamic LDS bytes of a launch
    // builds of the kernel: [symmetric block-Jacobi form][FP64 refinement]
    const void* fn[2][2];
    void (*launch[2][2])(const FusedParams&, dim3, size_t, hipStream_t);
    // the pipelined two-wave form ([symmetric form]; no refinement), when built
    const void* pipe_fn[2] = {nullptr, nullptr};
    void (*pipe_launch[2])(const FusedParams&, dim3, size_t, hipStream_t) = {nullptr, nullptr};
    size_t (*pipe_lds)(bool split, int refresh_every) = nullptr;
};

void register_f64(std::vector<KernelEntry>& v);
void register_f32(std::vector<KernelEntry>& v);
void register_bf16(std::vector<KernelEntry>& v);
void register_f16(std::vector<KernelEntry>& v);
void register_f8(std::vector<KernelEntry>& v);
void register_k128_f8(std::vector<KernelEntry>& v);
void register_k128_f16(std::vector<KernelEntry>& v);
void register_k64w_f16(std::vector<KernelEntry>& v);
void register_k64w_f64(std::vector<KernelEntry>& v);
void register_slab64(std::vector<KernelEntry>& v);
void register_slab64_f64(std::vector<KernelEntry>& v);
void register_slab128(std::vector<KernelEntry>& v);

// default waves per channel for a padded K and operand format: one wave holds
// the whole iterate (K/4 complex entries per lane) except where the FP64
// vectors would not fit the register file, and at K = 128 (two waves, K/8
// entries).  Other wave counts are registered beside the default where built
// (each wave owns K/(4 NW) entries per lane, so a Jacobi block must fit them).
constexpr int waves_for(int KP, int FMT) { return ((FMT == F64 && KP >= 64) || KP >= 128) ? 2 : 1; }

template <int KP, int NW, int FMT, int LB, bool SP, bool RF, typename IOT>
void set_build(KernelEntry& e) {
    e.fn[SP][RF] = reinterpret_cast<const void*>(&fused_kernel<KP, NW, FMT, LB, SP, RF, IOT>);
    e.launch[SP][RF] = [](const FusedParams& p, dim3 grid, size_t lds, hipStream_t s) {
        hipLaunchKernelGGL((fused_kernel<KP, NW, FMT, LB, SP, RF, IOT>), grid, dim3(64 * NW), lds, s, p);
    };
}

// LB = 0 builds only the plain form (the symmetric slot repeats it)
template <int KP, int FMT, int LB, typename IOT, int NW = waves_for(KP, FMT)>
void add_entry(std::vector<KernelEntry>& v) {
    static_assert(LB == 0 || (KP / (4 * NW)) % LB == 0, "a Jacobi block lies in one lane's entries");
    using C = Cfg<KP, NW, FMT, LB>;
    KernelEntry e;
    e.KP = KP; e.NW = NW; e.FMT = FMT; e.LB = LB;
    e.io_c64 = sizeof(IOT) == 4 ? 1 : 0;
    e.arow = C::AROW ? 1 : 0;
    e.lds = [](bool sp, bool r, int f) -> size_t { return C::lds(LB > 0 && sp, r, f); };
    set_build<KP, NW, FMT, LB, false, false, IOT>(e);
    // refinement builds only where their LDS layout fits (160 KiB)
    if constexpr (C::lds_general(false, true, 0) <= 160 * 1024) set_build<KP, NW, FMT, LB, false, true, IOT>(e);
    else { e.fn[0][1] = nullptr; e.launch[0][1] = nullptr; }
    if constexpr (LB > 0 && !C::AROW) {               // the symmetric form needs the u_W Gram in LDS
        set_build<KP, NW, FMT, LB, true, false, IOT>(e);
        set_build<KP, NW, FMT, LB, true, true, IOT>(e);
    } else if constexpr (LB > 0) {
        e.fn[1][0] = e.fn[1][1] = nullptr;
        e.launch[1][0] = e.launch[1][1] = nullptr;
    } else {
        e.fn[1][0] = e.fn[0][0]; e.fn[1][1] = e.fn[0][1];
        e.launch[1][0] = e.launch[0][0]; e.launch[1][1] = e.launch[0][1];
    }
    if constexpr (NW == 1 && KP <= 32) {
        e.pipe_lds = [](bool sp, int f) -> size_t { return PipeCfg<KP, FMT, LB>::lds(LB > 0 && sp, f); };
        e.pipe_fn[0] = reinterpret_cast<const void*>(&pipe_kernel<KP, FMT, LB, false, IOT>);
        e.pipe_launch[0] = [](const FusedParams& p, dim3 grid, size_t lds, hipStream_t s) {
            hipLaunchKernelGGL((pipe_kernel<KP, FMT, LB, false, IOT>), grid, dim3(128), lds, s, p);
        };
        if constexpr (LB > 0) {
            e.pipe_fn[1] = reinterpret_cast<const void*>(&pipe_kernel<KP, FMT, LB, true, IOT>);
            e.pipe_launch[1] = [](const FusedParams& p, dim3 grid, size_t lds, hipStream_t s) {
                hipLaunchKernelGGL((pipe_kernel<KP, FMT, LB, true, IOT>), grid, dim3(128), lds, s, p);
            };
        } else {
            e.pipe_fn[1] = e.pipe_fn[0];
            e.pipe_launch[1] = e.pipe_launch[0];
        }
    }
    v.push_back(e);
}

// the slab kernel of (KP, FMT, LB): builds [symmetric form][FP64 refresh]
// (FP64 operands: no refresh build)
template <int KP, int FMT, int LB, bool SP, bool RF, typename IOT>
void set_slab(KernelEntry& e) {
    e.fn[SP][RF] = reinterpret_cast<const void*>(&slab_kernel<KP, FMT, LB, SP, RF, IOT>);
    e.launch[SP][RF] = [](const FusedParams& p, dim3 grid, size_t lds, hipStream_t s) {
        hipLaunchKernelGGL((slab_kernel<KP, FMT, LB, SP, RF, IOT>), grid, dim3(64 * (KP / 16)), lds, s, p);
    };
}

template <int KP, int FMT, int LB, typename IOT>
void add_slab_entry(std::vector<KernelEntry>& v) {
    using C = SlabCfg<KP, FMT, LB>;
    KernelEntry e;
    e.KP = KP; e.NW = C::NW; e.FMT = FMT; e.LB = LB;
    e.io_c64 = sizeof(IOT) == 4 ? 1 : 0;
    e.kind = 1;
    e.arow = 0;
    e.lds = [](bool sp, bool, int f) -> size_t { return C::lds(sizeof(IOT) * 2, LB > 0 && sp, f > 0); };
    // refresh builds: FP32 and reduced formats at K = 64, and at K = 128 with L = 16
    constexpr bool RFB = FMT != F64 && (KP == 64 || LB == 16);
    if constexpr (LB >= 8) {                           // L = 8 and 16: the symmetric form only
        e.fn[0][0] = e.fn[0][1] = nullptr;
        e.launch[0][0] = e.launch[0][1] = nullptr;
    } else {
        set_slab<KP, FMT, LB, false, false, IOT>(e);
        if constexpr (RFB) set_slab<KP, FMT, LB, false, true, IOT>(e);
        else { e.fn[0][1] = nullptr; e.launch[0][1] = nullptr; }
    }
    if constexpr (LB > 0) {
        set_slab<KP, FMT, LB, true, false, IOT>(e);
        if constexpr (RFB) set_slab<KP, FMT, LB, true, true, IOT>(e);
        else { e.fn[1][1] = nullptr; e.launch[1][1] = nullptr; }
    } else {
        e.fn[1][0] = e.fn[0][0]; e.fn[1][1] = e.fn[0][1];
        e.launch[1][0] = e.launch[0][0]; e.launch[1][1] = e.launch[0][1];
    }
    v.push_back(e);
}

#define FPCG_SLAB_IO(KP_, FMT_, LB_)            \
    add_slab_entry<KP_, FMT_, LB_, float>(v);    \
    add_slab_entry<KP_, FMT_, LB_, double>(v)

#define FPCG_ENTRY(KP_, FMT_, LB_, IOT_) add_entry<KP_, FMT_, LB_, IOT_>(v)

#define FPCG_ENTRIES_IO(KP_, FMT_, LB_) \
    FPCG_ENTRY(KP_, FMT_, LB_, float);  \
    FPCG_ENTRY(KP_, FMT_, LB_, double)

// the same with NW_ waves per channel
#define FPCG_ENTRIES_IO_NW(KP_, FMT_, LB_, NW_)    \
    add_entry<KP_, FMT_, LB_, float, NW_>(v);    \
    add_entry<KP_, FMT_, LB_, double, NW_>(v)

}  // namespace fpcg
