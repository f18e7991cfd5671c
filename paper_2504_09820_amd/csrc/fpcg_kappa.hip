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
// over its recorded columns.  Two lanes per column search together
// (three sections per round), so a wave holds eight channels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fpcg_host.hpp"
#include "fpcg_fused.hpp"

namespace fpcg {

namespace {

constexpr int KMAXM = 32;      // steps used: the first min(I, 32)

// number of eigenvalues below x of the tridiagonal (d, e2) of order MR:
// rows past a column's own order carry a huge diagonal and no coupling, so
// their pivots are positive and never counted (no branches: MR is the
// compile-time row count, fully unrolled)
template <int MR>
__device__ __forceinline__ int sturm_below(const float (&d)[MR], const float (&e2)[MR], float x) {
    float q = d[0] - x;
    int c = q < 0.f;
#pragma unroll
    for (int i = 1; i < MR; ++i) {
        // a zero pivot gives an infinite next one (counted negative), whose
        // reciprocal is zero: the usual continuation of the recurrence
        q = (d[i] - x) - e2[i] * __builtin_amdgcn_rcpf(q);
        c += q < 0.f;
    }
    return c;
}

// Lanes: [channel of the wave][recorded column (KAPPA_COLS)][probe (NP)].
// The NP lanes of a column evaluate NP Sturm counts at once and shrink the
// bracket of an extreme eigenvalue by NP + 1 per round (multisection).
constexpr int NP = 2;
static_assert(64 % (KAPPA_COLS * NP) == 0, "whole channels per wave");
constexpr int CH_PER_WAVE = 64 / (KAPPA_COLS * NP);

// the probe lanes' flags of this lane's column -> index of the first probe
// whose flag is set (NP if none); uniform over the column's lanes
__device__ __forceinline__ int first_set(bool f, int lane) {
    const uint64_t m = __ballot(f);
    const uint32_t g = (uint32_t)(m >> (lane & ~(NP - 1))) & ((1u << NP) - 1u);
    return g ? __builtin_ctz(g) : NP;
}

// kappa estimate of this lane's column (NaN: no step) from its first
// mu <= MR recorded steps; p is the lane's probe
template <int MR>
__device__ float column_kappa(const float* h, int mu, bool valid, int p, int lane) {
    float a[MR], b[MR];
#pragma unroll
    for (int i = 0; i < MR; ++i) {                    // every load in flight at once
        const bool in = valid && i < mu;
        a[i] = in ? h[2 * i] : 0.f;
        b[i] = in ? h[2 * i + 1] : 0.f;
    }
    // (reciprocals by v_rcp_f32: the estimate needs a few digits, not ulps)
    float d[MR], e2[MR];
    int m = 0;
    bool go = valid;
    float ra_prev = 0.f, bp = 0.f;
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        go = go && a[i] > 0.f && __builtin_isfinite(a[i]);
        if (go) m = i + 1;
        const float ra = __builtin_amdgcn_rcpf(a[i]);
        d[i] = go ? ra + bp * ra_prev : 1e30f;
        e2[i] = go ? bp * ra_prev * ra_prev : 0.f;
        ra_prev = ra;
        bp = __builtin_isfinite(b[i]) ? b[i] : 0.f;
    }
    if (m == 0) d[0] = 1.f;                           // keeps the probes finite; the result is NaN
    float dmax = d[0], dmin = d[0], glo = INFINITY, ghi = -INFINITY;
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        if (i < m) {
            const float el = i ? __builtin_sqrtf(e2[i]) : 0.f;
            const float er = (i + 1 < MR && i + 1 < m) ? __builtin_sqrtf(e2[i + 1 < MR ? i + 1 : i]) : 0.f;
            dmax = fmaxf(dmax, d[i]);
            dmin = fminf(dmin, d[i]);
            glo = fminf(glo, d[i] - el - er);
            ghi = fmaxf(ghi, d[i] + el + er);
        }
    }
    // lambda_max in [max d, Gershgorin bound]: 9 rounds of 3 sections (1 / 19683)
    float lo = dmax, hi = fmaxf(ghi, dmax);
    for (int s = 0; s < 9; ++s) {
        const float w = (hi - lo) * (1.f / (NP + 1));
        const int j = first_set(sturm_below<MR>(d, e2, lo + w * (p + 1)) >= m, lane);
        const float nlo = lo + w * j, nhi = (j == NP) ? hi : lo + w * (j + 1);
        lo = nlo;
        hi = nhi;
    }
    const float lmax = 0.5f * (lo + hi);
    // lambda_min in (Gershgorin bound, min d], sections equal on a log scale:
    // 11 rounds (1 / 177147 of the log range)
    float hi2 = dmin, lo2 = (glo > 0.f) ? glo : dmin * 0x1p-30f;
    const bool below = first_set(sturm_below<MR>(d, e2, lo2) >= 1, lane) == 0;   // all probes agree
    for (int s = 0; s < 11; ++s) {
        const float t = __log2f(hi2 / lo2) * (1.f / (NP + 1));
        const int j = first_set(sturm_below<MR>(d, e2, lo2 * exp2f(t * (p + 1))) >= 1, lane);
        const float nlo = lo2 * exp2f(t * j), nhi = (j == NP) ? hi2 : lo2 * exp2f(t * (j + 1));
        lo2 = nlo;
        hi2 = nhi;
    }
    if (m == 0) return __builtin_nanf("");
    if (below) return lmax / (dmin * 0x1p-30f);       // below the searched range: a lower estimate
    return lmax / sqrtf(lo2 * hi2);
}

template <int MR>
__global__ __launch_bounds__(64) void kappa_kernel(const float* __restrict__ hist, int64_t n, int R, int iters,
                                                   const int32_t* __restrict__ chan_idx, int64_t B,
                                                   float* __restrict__ kappa) {
    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x * (int64_t)CH_PER_WAVE + lane / (KAPPA_COLS * NP);
    const int c = (lane / NP) % KAPPA_COLS, p = lane % NP, nrec = R < KAPPA_COLS ? R : KAPPA_COLS;
    const bool valid = item < n && c < nrec;
    // every lane of the wave runs the same rounds (the probes' ballots)
    float k = column_kappa<MR>(valid ? hist + ((size_t)item * nrec + c) * iters * 2 : hist, iters < MR ? iters : MR,
                               valid, p, lane);
    if (!valid) k = __builtin_nanf("");
    // largest over the channel's columns (NaN-ignoring maximum)
#pragma unroll
    for (int o = NP; o < KAPPA_COLS * NP; o <<= 1) k = fmaxf(k, __shfl_xor(k, o, KAPPA_COLS * NP));
    if (item < n && c == 0 && p == 0) {
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
        // rows of the tridiagonal: the steps used, rounded up to 8, 16 or 32
        const dim3 g((unsigned)((n + CH_PER_WAVE - 1) / CH_PER_WAVE));
        if (iters <= 8) hipLaunchKernelGGL(kappa_kernel<8>, g, dim3(64), 0, stream, hist, n, R, iters, chan_idx, B, kappa);
        else if (iters <= 16) hipLaunchKernelGGL(kappa_kernel<16>, g, dim3(64), 0, stream, hist, n, R, iters, chan_idx, B, kappa);
        else hipLaunchKernelGGL(kappa_kernel<KMAXM>, g, dim3(64), 0, stream, hist, n, R, iters, chan_idx, B, kappa);
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(FPCG_E_DEVICE, "kappa kernel launch: %s", hipGetErrorString(err));
    return FPCG_OK;
}

}  // namespace fpcg
