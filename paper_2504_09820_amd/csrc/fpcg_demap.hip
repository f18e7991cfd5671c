// Soft output after detection: max-log LLRs of Gray square-QAM symbols from
// the detector's estimate x_hat and each user's effective gain mu (the
// fpcg_detect_ex gain output).
//
// Model of the LMMSE estimate with unit-energy symbols (eq. inversion):
// x_hat = mu s + e, e of variance nu^2 = mu (1 - mu).  The max-log LLR of a
// label bit is (D1 - D0) / nu^2, D_v the smallest |x_hat - mu s|^2 over the
// points whose bit is v.  The label is (gray(j_I) << log2 m) | gray(j_Q), so
// the bits of one axis depend on that axis alone and the other axis's term
// cancels in D1 - D0: each axis is an m-level PAM problem, done here by
// comparing the m distances (m <= 16, a compile-time count, so every level's
// Gray bits are constants).
//
// HBM-bound: per symbol the estimate is read once (8 or 16 bytes), the gain
// once per R symbols, and log2(Q) floats are written.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fpcg_host.hpp"

namespace fpcg {

namespace {

template <int M> constexpr int log2_of() { return M <= 1 ? 0 : 1 + log2_of<M / 2>(); }

// LLRs of the BA = log2 M bits of one axis, most significant first, into o
template <int M, typename T>
__device__ __forceinline__ void axis_llr(T v, T c, T s, float* o) {
    constexpr int BA = log2_of<M>();
    T d0[BA], d1[BA];
#pragma unroll
    for (int p = 0; p < BA; ++p) { d0[p] = INFINITY; d1[p] = INFINITY; }
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const T e = fma(-c, (T)(2 * j - (M - 1)), v);   // c = mu / nu_Q: level j scaled by the gain
        const T d = e * e;
        const int gj = j ^ (j >> 1);
#pragma unroll
        for (int p = 0; p < BA; ++p) {
            if ((gj >> p) & 1) d1[p] = fmin(d1[p], d);
            else d0[p] = fmin(d0[p], d);
        }
    }
#pragma unroll
    for (int p = 0; p < BA; ++p) {
        const T diff = d1[p] - d0[p];
        // ties give 0 also where s is infinite (mu = 0 or 1); NaN stays NaN
        o[BA - 1 - p] = (float)(diff == (T)0 ? (T)0 : diff * s);
    }
}

// an LLR as a saturated 8-bit integer: round(llr * scale) to nearest even,
// clamped to [-127, 127]; NaN (no decision possible) becomes 0
__device__ __forceinline__ uint32_t quant8(float v, float scale) {
    float t = v * scale;
    t = (t != t) ? 0.f : t;
    t = fminf(fmaxf(__builtin_rintf(t), -127.f), 127.f);
    return (uint32_t)(uint8_t)(int8_t)(int)t;
}

// IT: the symbol index type (32-bit where n allows: cheaper gain index i / R);
// OT: float LLRs, or int8_t quantised with qscale
template <int M, typename T, typename IT, typename OT>
__global__ __launch_bounds__(256) void demap_kernel(IT n, IT R, const T* __restrict__ x,
                                                    const float* __restrict__ gain, T inv_nu,
                                                    OT* __restrict__ llr, float qscale) {
    constexpr int NB = 2 * log2_of<M>();
    for (IT i = blockIdx.x * (IT)blockDim.x + threadIdx.x; i < n; i += (IT)gridDim.x * blockDim.x) {
        // a non-finite component makes the whole symbol NaN (as its 2-D
        // distances are), not only that axis's bits
        T xr = x[2 * (int64_t)i], xi = x[2 * (int64_t)i + 1];
        const T poison = (xr - xr) + (xi - xi);
        xr += poison;
        xi += poison;
        T mu = (T)gain[i / R];
        mu = mu < (T)0 ? (T)0 : (mu > (T)1 ? (T)1 : mu);          // NaN passes through
        const T nu2 = mu * ((T)1 - mu);
        const T s = nu2 > (T)0 ? (T)1 / nu2 : (nu2 == (T)0 ? (T)INFINITY : (T)NAN);
        const T c = mu * inv_nu;
        float o[NB];
        axis_llr<M, T>(xr, c, s, o);
        axis_llr<M, T>(xi, c, s, o + NB / 2);
        OT* dst = llr + (int64_t)i * NB;
        if constexpr (sizeof(OT) == 1) {
            // NB bytes per symbol: one 2-, 4- or 8-byte store, or three 2-byte stores for NB = 6
            uint32_t q[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) q[k] = quant8(o[k], qscale);
            if constexpr (NB == 8) {
                const uint32_t lo = q[0] | (q[1] << 8) | (q[2] << 16) | (q[3] << 24);
                const uint32_t hi = q[4] | (q[5] << 8) | (q[6] << 16) | (q[7] << 24);
                *reinterpret_cast<uint2*>(dst) = make_uint2(lo, hi);
            } else if constexpr (NB == 4) {
                *reinterpret_cast<uint32_t*>(dst) = q[0] | (q[1] << 8) | (q[2] << 16) | (q[3] << 24);
            } else {
#pragma unroll
                for (int k = 0; k < NB; k += 2) *reinterpret_cast<uint16_t*>(dst + k) = (uint16_t)(q[k] | (q[k + 1] << 8));
            }
        } else if constexpr (NB % 4 == 0) {
#pragma unroll
            for (int k = 0; k < NB; k += 4) *reinterpret_cast<float4*>(dst + k) = make_float4(o[k], o[k + 1], o[k + 2], o[k + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < NB; k += 2) *reinterpret_cast<float2*>(dst + k) = make_float2(o[k], o[k + 1]);
        }
    }
}

unsigned demap_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return (unsigned)b;
}

template <typename T, typename IT, typename OT>
void launch_demap(hipStream_t s, int m, IT n, IT R, const void* x, const float* gain, double inv_nu, OT* llr,
                  float qscale) {
    const dim3 g(demap_grid(n)), b(256);
    const T* xp = static_cast<const T*>(x);
    const T in = (T)inv_nu;
    switch (m) {
        case 2: hipLaunchKernelGGL((demap_kernel<2, T, IT, OT>), g, b, 0, s, n, R, xp, gain, in, llr, qscale); break;
        case 4: hipLaunchKernelGGL((demap_kernel<4, T, IT, OT>), g, b, 0, s, n, R, xp, gain, in, llr, qscale); break;
        case 8: hipLaunchKernelGGL((demap_kernel<8, T, IT, OT>), g, b, 0, s, n, R, xp, gain, in, llr, qscale); break;
        default: hipLaunchKernelGGL((demap_kernel<16, T, IT, OT>), g, b, 0, s, n, R, xp, gain, in, llr, qscale); break;
    }
}

// argument checks shared by both entry points, then the launch
template <typename OT>
fpcg_status demap_entry(void* stream, int64_t n, int32_t R, const void* x, int32_t x_c64, const float* gain,
                        int32_t qam_order, OT* llr, float qscale, int align) {
    if (n < 0) return fail(FPCG_E_INVAL, "n=%lld < 0", (long long)n);
    if (R < 1) return fail(FPCG_E_INVAL, "R=%d < 1", R);
    if (!(qam_order == 4 || qam_order == 16 || qam_order == 64 || qam_order == 256))
        return fail(FPCG_E_INVAL, "qam_order=%d", qam_order);
    if (!(qscale > 0.f) || !std::isfinite(qscale)) return fail(FPCG_E_INVAL, "scale must be finite and positive");
    if (n == 0) return FPCG_OK;
    if (!x || !gain || !llr) return fail(FPCG_E_INVAL, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(llr) % align) return fail(FPCG_E_INVAL, "llr must be %d-byte aligned", align);
    const int m = (int)std::lround(std::sqrt((double)qam_order));
    const double inv_nu = 1.0 / std::sqrt(2.0 * (qam_order - 1) / 3.0);
    hipStream_t s = (hipStream_t)stream;
    // 32-bit indices while the grid-stride loop cannot pass 2^32
    const bool narrow = n <= (int64_t)UINT32_MAX - (int64_t)65535 * 256;
    if (narrow) {
        if (x_c64) launch_demap<float, uint32_t, OT>(s, m, (uint32_t)n, (uint32_t)R, x, gain, inv_nu, llr, qscale);
        else launch_demap<double, uint32_t, OT>(s, m, (uint32_t)n, (uint32_t)R, x, gain, inv_nu, llr, qscale);
    } else {
        if (x_c64) launch_demap<float, int64_t, OT>(s, m, n, (int64_t)R, x, gain, inv_nu, llr, qscale);
        else launch_demap<double, int64_t, OT>(s, m, n, (int64_t)R, x, gain, inv_nu, llr, qscale);
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(FPCG_E_DEVICE, "demap launch: %s", hipGetErrorString(err));
    return FPCG_OK;
}

}  // namespace

}  // namespace fpcg

using namespace fpcg;

extern "C" fpcg_status fpcg_demap_maxlog(void* stream, int64_t n, int32_t R, const void* x, int32_t x_c64,
                                         const float* gain, int32_t qam_order, float* llr) {
    clear_error();
    return demap_entry<float>(stream, n, R, x, x_c64, gain, qam_order, llr, 1.f, 16);
}

extern "C" fpcg_status fpcg_demap_maxlog_i8(void* stream, int64_t n, int32_t R, const void* x, int32_t x_c64,
                                            const float* gain, int32_t qam_order, float scale, int8_t* llr) {
    clear_error();
    return demap_entry<int8_t>(stream, n, R, x, x_c64, gain, qam_order, llr, scale, 8);
}
