// Internal host-side declarations shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <tuple>
#include <vector>

#include "fpcg.h"

// shape class of a launch: padded K, operand format, Jacobi block size,
// symmetric form, refresh on, complex64 I/O, several blocks of received vectors
using fpcg_tune_key = std::tuple<int, int, int, int, int, int, int>;

// (Nbs, K, block size) of a workload class whose expected condition number
// the context holds for the precision heuristic
using fpcg_kappa_key = std::tuple<int, int, int>;

struct fpcg_ctx {
    int device = 0;
    size_t budget = 0;
    int launch_form = FPCG_LAUNCH_AUTO;
    std::map<fpcg_tune_key, int> tuned;   // launch form chosen by fpcg_autotune per shape class
    std::map<fpcg_kappa_key, double> kappa;   // E{kappa} per workload class (fpcg_expected_kappa / fpcg_set_kappa)
};

namespace fpcg {

struct Plan {
    int KP = 0, FMT = 0, LB = 0;
    fpcg_schedule sched{};
};

fpcg_status fail(fpcg_status st, const char* fmt, ...);
void clear_error();

fpcg_status check_args(int64_t B, int32_t Nbs, int32_t K, int32_t R, int32_t qam, int32_t iters, int32_t L,
                       const fpcg_schedule* s, Plan* plan);

// the schedule a NULL schedule stands for: the precision heuristic's format
// for the context's E{kappa} of (Nbs, K, L) (fpcg_policy.hip)
fpcg_status resolve_schedule(const fpcg_ctx* ctx, int64_t B, int32_t Nbs, int32_t K, int32_t R, int32_t qam,
                             int32_t iters, int32_t L, const fpcg_schedule* s, fpcg_schedule* out);
// parse / print the context's table of tuned launch forms and E{kappa}
fpcg_status parse_tune_table(const char* text, fpcg_ctx* ctx);

using TuneKey = fpcg_tune_key;
TuneKey tune_key(const Plan& plan, int32_t R, int32_t io_c64);
// launch forms built for a plan (FPCG_LAUNCH_FUSED first)
std::vector<int> launch_forms(const Plan& plan, int32_t R, int32_t io_c64);
// a launch over a subset of the batch (chan_idx: n indices, NULL = all B) and
// an optional record of the CG coefficients (n x R x iters x 2 floats)
struct LaunchExtra {
    const int32_t* chan_idx = nullptr;
    int64_t n = 0;
    float* ab_hist = nullptr;
    float* gain = nullptr;
    void* gram_out = nullptr;    // step 1 only: the Gram and matched filter in u_W
    void* mf_out = nullptr;
    void* T_out = nullptr;       // the block-Jacobi factor, written / read in place of its factorisation
    const void* T_in = nullptr;
};
// one launch in the given form (FPCG_LAUNCH_FUSED or FPCG_LAUNCH_PIPELINED;
// a launch with extras always runs fused)
fpcg_status launch_detect_form(const fpcg_ctx* ctx, hipStream_t stream, const Plan& plan, int form, int64_t B,
                               int32_t Nbs, int32_t K, int32_t R, const void* H, const void* Y, int32_t io_c64,
                               const double* sigma2, int32_t qam, int32_t iters, void* xhat, uint8_t* labels,
                               uint32_t* flags, const LaunchExtra* ex = nullptr);
// per-channel kappa estimates from a coefficient record (fpcg_kappa.hip)
fpcg_status launch_kappa(hipStream_t stream, const float* hist, int64_t n, int32_t R, int32_t iters,
                         const int32_t* chan_idx, int64_t B, float* kappa);

fpcg_status launch_detect(const fpcg_ctx* ctx, hipStream_t stream, const Plan& plan, int64_t B, int32_t Nbs, int32_t K,
                          int32_t R, const void* H, const void* Y, int32_t io_c64, const double* sigma2, int32_t qam,
                          int32_t iters, void* xhat, uint8_t* labels, uint32_t* flags);

}  // namespace fpcg
