// Launch-form autotuner (fpcg_autotune in fpcg.h).
//
// For one shape class -- padded K, operand format, Jacobi block size,
// block-Jacobi form, refresh on or off, I/O element type, one or several
// blocks of received vectors -- every launch form built for it is timed on
// synthetic inputs of the caller's size, with the candidates interleaved so
// that clock drift under sustained load falls on all of them alike.  The
// fastest form is recorded in the context and used by FPCG_LAUNCH_AUTO.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "fpcg_host.hpp"

using namespace fpcg;

namespace {

// deterministic inputs: the element index through MurmurHash3's 32-bit
// finaliser, mapped to [-a, a)
__global__ void fill_hash(float* p, int64_t n, uint32_t seed, float a) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 0x9E3779B1u ^ seed;
        h ^= h >> 16; h *= 0x85EBCA6Bu; h ^= h >> 13; h *= 0xC2B2AE35u; h ^= h >> 16;
        p[i] = a * ((float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f);
    }
}
__global__ void fill_hash64(double* p, int64_t n, uint32_t seed, double a) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 0x9E3779B1u ^ seed;
        h ^= h >> 16; h *= 0x85EBCA6Bu; h ^= h >> 13; h *= 0xC2B2AE35u; h ^= h >> 16;
        p[i] = a * ((double)(h >> 8) * (1.0 / 8388608.0) - 1.0);
    }
}
__global__ void fill_const64(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

}  // namespace

extern "C" fpcg_status fpcg_autotune(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R,
                                     int32_t io_c64, int32_t qam_order, int32_t iters, int32_t block_L,
                                     const fpcg_schedule* sched, int32_t reps, int32_t* chosen_form) {
    clear_error();
    if (!ctx) return fail(FPCG_E_INVAL, "ctx is NULL");
    if (reps < 1 || reps > 1000) return fail(FPCG_E_INVAL, "reps=%d must be in [1, 1000]", reps);
    fpcg_schedule rs;
    fpcg_status st = resolve_schedule(ctx, B, Nbs, K, R, qam_order, iters, block_L, sched, &rs);
    if (st != FPCG_OK) return st;
    Plan plan;
    st = check_args(B, Nbs, K, R, qam_order, iters, block_L, &rs, &plan);
    if (st != FPCG_OK) return st;
    if (B < 1) return fail(FPCG_E_INVAL, "B=%lld: nothing to time", (long long)B);
    const std::vector<int> forms = launch_forms(plan, R, io_c64);
    const TuneKey key = tune_key(plan, R, io_c64);
    if (forms.size() < 2) {
        ctx->tuned[key] = forms.empty() ? FPCG_LAUNCH_FUSED : forms[0];
        if (chosen_form) *chosen_form = ctx->tuned[key];
        return FPCG_OK;
    }
    int prev_dev = -1;
    (void)hipGetDevice(&prev_dev);
    (void)hipSetDevice(ctx->device);
    struct Restore { int d; ~Restore() { if (d >= 0) (void)hipSetDevice(d); } } restore{prev_dev};
    hipStream_t s = (hipStream_t)stream;
    const size_t el = io_c64 ? 8 : 16;
    const size_t nh = (size_t)B * Nbs * K, ny = (size_t)B * Nbs * R, nx = (size_t)B * K * R;
    void *dH = nullptr, *dY = nullptr, *dX = nullptr;
    double* dS = nullptr;
    uint8_t* dL = nullptr;
    uint32_t* dF = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        if (dH) (void)hipFree(dH);
        if (dY) (void)hipFree(dY);
        if (dX) (void)hipFree(dX);
        if (dS) (void)hipFree(dS);
        if (dL) (void)hipFree(dL);
        if (dF) (void)hipFree(dF);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&dH, nh * el) != hipSuccess || hipMalloc(&dY, ny * el) != hipSuccess ||
        hipMalloc(&dX, nx * el) != hipSuccess || hipMalloc((void**)&dS, B * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&dL, nx) != hipSuccess || hipMalloc((void**)&dF, B * sizeof(uint32_t)) != hipSuccess) {
        cleanup();
        return fail(FPCG_E_NOMEM, "autotune buffers (%zu bytes of inputs)", (nh + ny) * el);
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(FPCG_E_DEVICE, "event creation failed");
    }
    // entries of H with variance about 1/Nbs, received vectors of unit scale
    const float ah = 1.7320508f / std::sqrt((float)Nbs);
    if (io_c64) {
        hipLaunchKernelGGL(fill_hash, dim3(blocks_for(2 * nh)), dim3(256), 0, s, (float*)dH, (int64_t)(2 * nh), 0x1234u, ah);
        hipLaunchKernelGGL(fill_hash, dim3(blocks_for(2 * ny)), dim3(256), 0, s, (float*)dY, (int64_t)(2 * ny), 0x5678u, 1.7320508f);
    } else {
        hipLaunchKernelGGL(fill_hash64, dim3(blocks_for(2 * nh)), dim3(256), 0, s, (double*)dH, (int64_t)(2 * nh), 0x1234u, (double)ah);
        hipLaunchKernelGGL(fill_hash64, dim3(blocks_for(2 * ny)), dim3(256), 0, s, (double*)dY, (int64_t)(2 * ny), 0x5678u, 1.7320508);
    }
    hipLaunchKernelGGL(fill_const64, dim3(blocks_for(B)), dim3(256), 0, s, dS, (int64_t)B, 0.01);
    std::vector<std::vector<float>> ms(forms.size());
    for (int rep = -2; rep < reps; ++rep) {            // two untimed rounds first
        for (size_t f = 0; f < forms.size(); ++f) {
            (void)hipEventRecord(e0, s);
            st = launch_detect_form(ctx, s, plan, forms[f], B, Nbs, K, R, dH, dY, io_c64, dS, qam_order, iters, dX, dL, dF);
            (void)hipEventRecord(e1, s);
            if (st != FPCG_OK) { cleanup(); return st; }
            if (hipEventSynchronize(e1) != hipSuccess) { cleanup(); return fail(FPCG_E_DEVICE, "autotune launch failed"); }
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (rep >= 0) ms[f].push_back(t);
        }
    }
    cleanup();
    int best = 0;
    float best_t = 0.f;
    for (size_t f = 0; f < forms.size(); ++f) {
        std::vector<float> v = ms[f];
        std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
        const float med = v[v.size() / 2];
        if (f == 0 || med < best_t) { best = (int)f; best_t = med; }
    }
    ctx->tuned[key] = forms[best];
    if (chosen_form) *chosen_form = forms[best];
    return FPCG_OK;
}
