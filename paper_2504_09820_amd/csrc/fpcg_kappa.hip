// Per-channel condition-number estimate from the CG coefficients of the
// detector's first solve (fpcg_detect_ex with a kappa output).
//
// The iterates of CG span a Krylov space whose Lanczos tridiagonal T follows
// from the step coefficients alone (a textbook identity, not the paper's):
//   T[0][0] = 1/alpha_1,  T[i][i] = 1/alpha_{i+1} + beta_i/alpha_i,
//   T[i-1][i]^2 = beta_i / alpha_i^2.
// Its eigenvalues (Ritz values) lie in the iteration matrix's spectrum (A,
// M_d A or A_bar), and its extreme ones converge first, so
// lambda_max(T)/lambda_min(T) is a per-channel lower estimate of the kappa
// that eq. heuristic / eq. heuristic_bj use in place of E{kappa}.  Each 16-lane
// group takes one channel, one lane per received-vector column; the extreme
// eigenvalues come from bisection on Sturm counts (LDL^T pivots), lambda_min
// on a logarithmic scale; the channel's estimate is the largest over its
// columns.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fpcg_host.hpp"

namespace fpcg {

namespace {

constexpr int KMAXM = 32;      // steps used: the first min(I, 32)

// number of eigenvalues of the tridiagonal (d, e2) below x
__device__ __forceinline__ int sturm_below(const float (&d)[KMAXM], const float (&e2)[KMAXM], int m, float x) {
    float q = d[0] - x;
    int c = q < 0.f;
#pragma unroll
    for (int i = 1; i < KMAXM; ++i) {
        if (i < m) {
            const float qq = (q == 0.f) ? 1e-30f : q;
            q = (d[i] - x) - e2[i] * __builtin_amdgcn_rcpf(qq);
            c += q < 0.f;
        }
    }
    return c;
}

// kappa estimate of one column from its recorded coefficients (NaN: no step)
__device__ float column_kappa(const float* h, int iters) {
    float d[KMAXM], e2[KMAXM];
    int m = 0;
    float a_prev = 1.f, b_prev = 0.f;
    bool go = true;
#pragma unroll
    for (int i = 0; i < KMAXM; ++i) {
        d[i] = 0.f;
        e2[i] = 0.f;
        if (go && i < iters) {
            const float a = h[2 * i], b = h[2 * i + 1];
            if (a > 0.f && __builtin_isfinite(a)) {
                d[i] = 1.f / a + (i ? b_prev / a_prev : 0.f);
                e2[i] = i ? b_prev / (a_prev * a_prev) : 0.f;
                a_prev = a;
                b_prev = __builtin_isfinite(b) ? b : 0.f;
                m = i + 1;
            } else {
                go = false;
            }
        }
    }
    if (m == 0) return __builtin_nanf("");
    float dmax = d[0], dmin = d[0], glo = INFINITY, ghi = -INFINITY;
#pragma unroll
    for (int i = 0; i < KMAXM; ++i) {
        if (i < m) {
            const float el = i ? sqrtf(e2[i]) : 0.f, er = (i + 1 < m) ? sqrtf(e2[i + 1]) : 0.f;
            dmax = fmaxf(dmax, d[i]);
            dmin = fminf(dmin, d[i]);
            glo = fminf(glo, d[i] - el - er);
            ghi = fmaxf(ghi, d[i] + el + er);
        }
    }
    // lambda_max in [max d, Gershgorin bound]
    float lo = dmax, hi = fmaxf(ghi, dmax);
    for (int s = 0; s < 16; ++s) {
        const float mid = 0.5f * (lo + hi);
        if (sturm_below(d, e2, m, mid) >= m) hi = mid; else lo = mid;
    }
    const float lmax = 0.5f * (lo + hi);
    // lambda_min in (Gershgorin bound, min d], geometric bisection
    float hi2 = dmin, lo2 = (glo > 0.f) ? glo : dmin * 0x1p-30f;
    if (sturm_below(d, e2, m, lo2) >= 1) return lmax / lo2;      // below the searched range: a lower estimate
    for (int s = 0; s < 18; ++s) {
        const float mid = sqrtf(lo2 * hi2);
        if (sturm_below(d, e2, m, mid) >= 1) hi2 = mid; else lo2 = mid;
    }
    return lmax / sqrtf(lo2 * hi2);
}

__global__ __launch_bounds__(64) void kappa_kernel(const float* __restrict__ hist, int64_t n, int R, int iters,
                                                   const int32_t* __restrict__ chan_idx, int64_t B,
                                                   float* __restrict__ kappa) {
    const int64_t item = blockIdx.x * 4ll + (threadIdx.x >> 4);
    const int n16 = threadIdx.x & 15;
    float k = __builtin_nanf("");
    if (item < n) {
        for (int c = n16; c < R; c += 16) {
            const float kc = column_kappa(hist + ((size_t)item * R + c) * iters * 2, iters);
            k = fmaxf(k, kc);                           // NaN-ignoring maximum
        }
    }
    // largest over the 16 lanes of the channel's group
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) k = fmaxf(k, __shfl_xor(k, o, 16));
    if (item < n && n16 == 0) {
        const int64_t ch = chan_idx ? chan_idx[item] : item;
        if (ch >= 0 && ch < B) kappa[ch] = k;
    }
}

__global__ void fill_nan(float* p, const int32_t* chan_idx, int64_t n, int64_t B) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ch = chan_idx ? chan_idx[i] : i;
        if (ch >= 0 && ch < B) p[ch] = __builtin_nanf("");
    }
}

}  // namespace

fpcg_status launch_kappa(hipStream_t stream, const float* hist, int64_t n, int32_t R, int32_t iters,
                         const int32_t* chan_idx, int64_t B, float* kappa) {
    if (n == 0) return FPCG_OK;
    if (iters == 0 || !hist) {
        const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(fill_nan, dim3(g), dim3(256), 0, stream, kappa, chan_idx, n, B);
    } else {
        hipLaunchKernelGGL(kappa_kernel, dim3((unsigned)((n + 3) / 4)), dim3(64), 0, stream, hist, n, R, iters,
                           chan_idx, B, kappa);
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(FPCG_E_DEVICE, "kappa kernel launch: %s", hipGetErrorString(err));
    return FPCG_OK;
}

}  // namespace fpcg
