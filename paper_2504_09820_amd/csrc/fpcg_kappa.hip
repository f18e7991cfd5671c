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
// that eq. heuristic / eq. heuristic_bj use in place of E{kappa}.  The first
// KAPPA_COLS received-vector columns are recorded (all share A; each explores
// it from its own right-hand side); one lane per recorded column, the
// extreme eigenvalues from bisection on Sturm counts (LDL^T pivots),
// lambda_min on a logarithmic scale; the channel's estimate is the largest
// over its recorded columns.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fpcg_host.hpp"
#include "fpcg_fused.hpp"

namespace fpcg {

namespace {

constexpr int KMAXM = 32;      // steps used: the first min(I, 32)

// number of eigenvalues below x of the tridiagonal (d, e2) padded to order
// mu (uniform over the wave): rows past a column's own order carry a huge
// diagonal and no coupling, so their pivots are positive and never counted
__device__ __forceinline__ int sturm_below(const float (&d)[KMAXM], const float (&e2)[KMAXM], int mu, float x) {
    float q = d[0] - x;
    int c = q < 0.f;
#pragma unroll
    for (int i = 1; i < KMAXM; ++i) {
        if (i >= mu) break;                           // uniform: a scalar branch
        const float qq = (q == 0.f) ? 1e-30f : q;
        q = (d[i] - x) - e2[i] * __builtin_amdgcn_rcpf(qq);
        c += q < 0.f;
    }
    return c;
}

// kappa estimate of one column from its recorded coefficients (NaN: no step);
// mu = min(iters, KMAXM) is the same for every lane
__device__ float column_kappa(const float* h, int mu) {
    float a[KMAXM], b[KMAXM];
#pragma unroll
    for (int i = 0; i < KMAXM; ++i) {                 // every load in flight at once
        a[i] = 0.f;
        b[i] = 0.f;
        if (i < mu) { a[i] = h[2 * i]; b[i] = h[2 * i + 1]; }
    }
    float d[KMAXM], e2[KMAXM];
    int m = 0;
    bool go = true;
#pragma unroll
    for (int i = 0; i < KMAXM; ++i) {
        go = go && i < mu && a[i] > 0.f && __builtin_isfinite(a[i]);
        if (go) m = i + 1;
        const float ap = i ? a[i - 1] : 1.f, bp = (i && __builtin_isfinite(b[i - 1])) ? b[i - 1] : 0.f;
        d[i] = go ? 1.f / a[i] + (i ? bp / ap : 0.f) : 1e30f;
        e2[i] = (go && i) ? bp / (ap * ap) : 0.f;
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
    for (int s = 0; s < 14; ++s) {
        const float mid = 0.5f * (lo + hi);
        if (sturm_below(d, e2, mu, mid) >= m) hi = mid; else lo = mid;
    }
    const float lmax = 0.5f * (lo + hi);
    // lambda_min in (Gershgorin bound, min d], geometric bisection
    float hi2 = dmin, lo2 = (glo > 0.f) ? glo : dmin * 0x1p-30f;
    if (sturm_below(d, e2, mu, lo2) >= 1) return lmax / lo2;      // below the searched range: a lower estimate
    for (int s = 0; s < 16; ++s) {
        const float mid = sqrtf(lo2 * hi2);
        if (sturm_below(d, e2, mu, mid) >= 1) hi2 = mid; else lo2 = mid;
    }
    return lmax / sqrtf(lo2 * hi2);
}

__global__ __launch_bounds__(64) void kappa_kernel(const float* __restrict__ hist, int64_t n, int R, int iters,
                                                   const int32_t* __restrict__ chan_idx, int64_t B,
                                                   float* __restrict__ kappa) {
    // KAPPA_COLS lanes per channel, one recorded column each
    const int64_t item = blockIdx.x * (64ll / KAPPA_COLS) + threadIdx.x / KAPPA_COLS;
    const int c = threadIdx.x % KAPPA_COLS, nrec = R < KAPPA_COLS ? R : KAPPA_COLS;
    float k = __builtin_nanf("");
    if (item < n && c < nrec)
        k = column_kappa(hist + ((size_t)item * nrec + c) * iters * 2, iters < KMAXM ? iters : KMAXM);
    // largest over the channel's lanes (NaN-ignoring maximum)
#pragma unroll
    for (int o = KAPPA_COLS / 2; o > 0; o >>= 1) k = fmaxf(k, __shfl_xor(k, o, KAPPA_COLS));
    if (item < n && c == 0) {
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
        const int64_t per_block = 64 / KAPPA_COLS;
        hipLaunchKernelGGL(kappa_kernel, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(64), 0, stream, hist,
                           n, R, iters, chan_idx, B, kappa);
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(FPCG_E_DEVICE, "kappa kernel launch: %s", hipGetErrorString(err));
    return FPCG_OK;
}

}  // namespace fpcg
