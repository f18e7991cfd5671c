// Host runtime behind include/fpcg.h: argument validation, variant dispatch,
// the stand-alone slicer / rounding kernels, the precision heuristic, error
// reporting and contexts.  The serving queue lives in fpcg_serve.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fpcg.h"
#include "fpcg_host.hpp"
#include "fpcg_registry.hpp"

namespace fpcg {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

fpcg_status fail(fpcg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void clear_error() { g_last_error.clear(); }

// ------------------------------------------------------------------ variant table
static std::vector<KernelEntry>& table() {
    static std::vector<KernelEntry> t;
    static std::once_flag once;
    std::call_once(once, [] {
        register_f64(t);
        register_f32(t);
        register_bf16(t);
        register_f16(t);
        register_f8(t);
        register_k128_f8(t);
        register_k128_f16(t);
        register_k64w_f16(t);
        register_k64w_f64(t);
        register_slab64(t);
        register_slab64_f64(t);
        register_slab128(t);
    });
    return t;
}

// the fused-kernel entry for (KP, FMT, LB, io) with NW waves per channel; NW = 0
// asks for the default wave count of that K and format
static const KernelEntry* find_entry(int KP, int FMT, int LB, int io_c64, int NW = 0) {
    const int want = NW ? NW : waves_for(KP, FMT);
    for (const auto& e : table())
        if (e.kind == 0 && e.KP == KP && e.FMT == FMT && e.LB == LB && e.io_c64 == io_c64 && e.NW == want) return &e;
    return nullptr;
}

// the slab-kernel entry for (KP, FMT, LB, io), if built
static const KernelEntry* find_slab(int KP, int FMT, int LB, int io_c64) {
    for (const auto& e : table())
        if (e.kind == 1 && e.KP == KP && e.FMT == FMT && e.LB == LB && e.io_c64 == io_c64) return &e;
    return nullptr;
}

// whether a built entry takes this schedule: its build exists (refinement for
// the fused kernel, the FP64 refresh for the slab kernel) and its LDS fits
static bool entry_takes(const KernelEntry* e, int LB, const fpcg_schedule& s) {
    if (!e) return false;
    const int sp = (LB > 0 && s.variant == 2) ? 1 : 0;
    const int b = e->kind == 1 ? (s.refresh_every > 0 ? 1 : 0) : (s.refine_steps > 0 ? 1 : 0);
    if (e->kind == 1 && s.refine_steps > 0) return false;
    if (e->kind == 0 && e->arow && s.refresh_every > 0) return false;   // no u_W Gram to refresh from
    if (!e->fn[sp][b]) return false;
    return e->lds(sp != 0, s.refine_steps > 0, s.refresh_every) <= 160 * 1024;
}

// wave counts built for (KP, FMT, LB, io), the default first
static std::vector<int> built_waves(int KP, int FMT, int LB, int io_c64) {
    std::vector<int> w;
    if (find_entry(KP, FMT, LB, io_c64)) w.push_back(waves_for(KP, FMT));
    for (const auto& e : table())
        if (e.KP == KP && e.FMT == FMT && e.LB == LB && e.io_c64 == io_c64 &&
            std::find(w.begin(), w.end(), e.NW) == w.end())
            w.push_back(e.NW);
    return w;
}

// smallest padded K with a compiled variant for (K, fmt, L)
static int pick_kp(int K, int FMT, int L) {
    static const int kps[] = {16, 32, 64, 128};
    for (int kp : kps) {
        if (kp < K) continue;
        const int sh = kp / (4 * waves_for(kp, FMT));
        if (FMT == F8 && kp < 32) continue;
        if (find_slab(kp, FMT, L, 1)) return kp;
        if (L > sh) continue;
        if (!find_entry(kp, FMT, L, 1)) continue;
        return kp;
    }
    return 0;
}

static bool valid_fmt(int f) { return f >= FPCG_F64 && f <= FPCG_F8E4M3; }

fpcg_status check_args(int64_t B, int32_t Nbs, int32_t K, int32_t R, int32_t qam, int32_t iters,
                       int32_t L, const fpcg_schedule* s, Plan* plan) {
    fpcg_schedule def = {FPCG_F64, FPCG_F64, FPCG_F64, FPCG_F64, 0, 0, 0};
    if (!s) s = &def;
    if (B < 0 || B > 0x7fffffffLL) return fail(FPCG_E_INVAL, "B=%lld out of range [0, 2^31-1]", (long long)B);
    if (Nbs < 1) return fail(FPCG_E_INVAL, "Nbs=%d must be >= 1", Nbs);
    if (K < 1) return fail(FPCG_E_INVAL, "K=%d must be >= 1", K);
    if (R < 1) return fail(FPCG_E_INVAL, "R=%d must be >= 1", R);
    if (!(qam == 4 || qam == 16 || qam == 64 || qam == 256))
        return fail(FPCG_E_INVAL, "qam_order=%d must be 4, 16, 64 or 256", qam);
    if (iters < 0) return fail(FPCG_E_INVAL, "iters=%d must be >= 0", iters);
    if (L < 0) return fail(FPCG_E_INVAL, "block_L=%d must be >= 0", L);
    if (L > 0 && K % L != 0) return fail(FPCG_E_INVAL, "block_L=%d does not divide K=%d", L, K);
    if (!valid_fmt(s->gram_op) || !valid_fmt(s->mv_op) || !valid_fmt(s->ip) || !valid_fmt(s->work))
        return fail(FPCG_E_INVAL, "schedule format out of range");
    if (s->refresh_every < 0) return fail(FPCG_E_INVAL, "refresh_every=%d must be >= 0", s->refresh_every);
    if (s->refine_steps < 0 || s->refine_steps > 16)
        return fail(FPCG_E_INVAL, "refine_steps=%d must be in [0, 16]", s->refine_steps);
    if (s->variant < 0 || s->variant > 2) return fail(FPCG_E_INVAL, "variant=%d must be 0, 1 or 2", s->variant);
    if (s->gram_op != s->mv_op)
        return fail(FPCG_E_UNSUPPORTED, "gram_op (%d) must equal mv_op (%d)", s->gram_op, s->mv_op);
    const int want_work = s->mv_op == FPCG_F64 ? FPCG_F64 : FPCG_F32;
    if (s->work != want_work || s->ip != want_work)
        return fail(FPCG_E_UNSUPPORTED, "work and ip must be %s for mv_op %d", want_work == FPCG_F64 ? "F64" : "F32", s->mv_op);
    if (K > 128) return fail(FPCG_E_UNSUPPORTED, "K=%d > 128 is not built", K);
    // per-channel byte ranges of H, Y and x_hat (complex128 at most) are 32-bit
    // buffer ranges below the out-of-range offset 2^31
    if ((int64_t)Nbs * std::max(K, R) * 16 >= (1LL << 31) || (int64_t)K * R * 16 >= (1LL << 31))
        return fail(FPCG_E_UNSUPPORTED, "Nbs=%d, K=%d, R=%d: one channel's data exceeds 2 GiB", Nbs, K, R);
    if (L != 0 && L != 4 && L != 8 && L != 16) return fail(FPCG_E_UNSUPPORTED, "block_L=%d not built (0, 4, 8, 16)", L);
    // map the public format enum to the kernel enum (identical values)
    const int fmt = s->mv_op;
    const int kp = pick_kp(K, fmt, L);
    if (!kp) return fail(FPCG_E_UNSUPPORTED, "no variant for K=%d fmt=%d L=%d", K, fmt, L);
    {
        // the layout does not depend on the I/O type; a shape class runs the
        // fused kernel where built for the schedule, else the slab kernel
        const KernelEntry* e = find_entry(kp, fmt, L, 1);
        const KernelEntry* es = find_slab(kp, fmt, L, 1);
        const int sp = (L > 0 && s->variant == 2) ? 1 : 0, ref = s->refine_steps > 0 ? 1 : 0;
        if (!entry_takes(e, L, *s) && !entry_takes(es, L, *s)) {
            if (e && e->arow && s->refresh_every > 0)
                return fail(FPCG_E_UNSUPPORTED, "K=%d: the FP64 refresh needs the u_W Gram, kept only for K <= 64", K);
            if (e && e->fn[sp][ref]) {
                const size_t lds = e->lds(sp != 0, ref != 0, s->refresh_every);
                return fail(FPCG_E_UNSUPPORTED, "this schedule at K=%d needs %zu bytes of LDS (160 KiB per workgroup)", K, lds);
            }
            return fail(FPCG_E_UNSUPPORTED, "K=%d: %s%s%s not built for this format", K,
                        sp ? "the symmetric block-Jacobi form" : "this form", ref ? " with refinement" : "",
                        s->refresh_every > 0 ? " with the FP64 refresh" : "");
        }
    }
    if (plan) {
        plan->KP = kp;
        plan->FMT = fmt;
        plan->LB = L;
        plan->sched = *s;
    }
    return FPCG_OK;
}

struct ScopedDevice {
    int prev = -1;
    explicit ScopedDevice(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~ScopedDevice() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// ------------------------------------------------------------------ static workspace
// The coefficient record of fpcg_detect_ex_static (callers that cannot
// allocate): a fixed device array, one copy on every GPU the library runs
// on, held until the process ends.  In host code `scratch` names a host-side
// stand-in; the address of a device's copy comes from hipGetSymbolAddress,
// taken once per device in fpcg_create with that device current.
static __device__ __align__(256) float scratch[FPCG_STATIC_SCRATCH_BYTES / sizeof(float)];

static std::mutex g_scratch_mu;
static std::map<int, float*> g_scratch_ptr;      // device -> its copy of `scratch`

static fpcg_status bind_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return FPCG_OK;
    void* ptr = nullptr;
    const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !ptr)
        return fail(FPCG_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(err));
    g_scratch_ptr[device] = static_cast<float*>(ptr);
    return FPCG_OK;
}

static float* scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

__global__ void zero_u32(uint32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0u;
}
// p[idx[i]] = 0 for the n indices in [0, B)
__global__ void zero_u32_at(uint32_t* p, const int32_t* idx, int64_t n, int64_t B) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = idx[i];
        if (c >= 0 && c < B) p[c] = 0u;
    }
}

static inline unsigned grid_for(int64_t n, int threads) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return (unsigned)b;
}

static int cu_count(int device) {
    static std::mutex mu;
    static std::map<int, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(device);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n < 1) n = 1;
    cache[device] = n;
    return n;
}

// resident two-wave workgroups per CU for a pipelined build and LDS size
static int pipe_occupancy(int device, const void* fn, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, size_t>, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_tuple(device, fn, lds);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 128, lds) != hipSuccess) nb = 0;
    cache[key] = nb;
    return nb;
}

TuneKey tune_key(const Plan& plan, int32_t R, int32_t io_c64) {
    return TuneKey(plan.KP, plan.FMT, plan.LB, (plan.LB > 0 && plan.sched.variant == 2) ? 1 : 0,
                   plan.sched.refresh_every > 0 ? 1 : 0, io_c64 ? 1 : 0, R > 16 ? 1 : 0);
}

std::vector<int> launch_forms(const Plan& plan, int32_t R, int32_t io_c64) {
    (void)R;
    std::vector<int> f;
    const int sp = (plan.LB > 0 && plan.sched.variant == 2) ? 1 : 0, ref = plan.sched.refine_steps > 0 ? 1 : 0;
    for (int nw : built_waves(plan.KP, plan.FMT, plan.LB, io_c64 ? 1 : 0)) {
        const KernelEntry* e = find_entry(plan.KP, plan.FMT, plan.LB, io_c64 ? 1 : 0, nw);
        if (!entry_takes(e, plan.LB, plan.sched)) continue;
        f.push_back(FPCG_LAUNCH_FUSED | (nw << FPCG_LAUNCH_WAVES_SHIFT));
    }
    const KernelEntry* e = find_entry(plan.KP, plan.FMT, plan.LB, io_c64 ? 1 : 0);
    if (entry_takes(e, plan.LB, plan.sched) && e->pipe_fn[sp] && !ref) f.push_back(FPCG_LAUNCH_PIPELINED);
    if (entry_takes(find_slab(plan.KP, plan.FMT, plan.LB, io_c64 ? 1 : 0), plan.LB, plan.sched))
        f.push_back(FPCG_LAUNCH_SLAB);
    return f;
}

fpcg_status launch_detect_form(const fpcg_ctx* ctx, hipStream_t stream, const Plan& plan, int form, int64_t B,
                               int32_t Nbs, int32_t K, int32_t R, const void* H, const void* Y, int32_t io_c64,
                               const double* sigma2, int32_t qam, int32_t iters, void* xhat, uint8_t* labels,
                               uint32_t* flags, const LaunchExtra* ex) {
    // waves per channel requested with the form; the default where that
    // count is not built for this shape class (or its layout would not fit)
    const int nw = form >> FPCG_LAUNCH_WAVES_SHIFT;
    form &= (1 << FPCG_LAUNCH_WAVES_SHIFT) - 1;
    const int sp = (plan.LB > 0 && plan.sched.variant == 2) ? 1 : 0;
    const int ref = plan.sched.refine_steps > 0 ? 1 : 0;
    const KernelEntry* e = nullptr;
    const bool extras_fused_only = ex && (ex->gain || ex->gram_out);   // outputs only the fused kernel writes
    if (nw && form == FPCG_LAUNCH_FUSED) {
        e = find_entry(plan.KP, plan.FMT, plan.LB, io_c64 ? 1 : 0, nw);
        if (!entry_takes(e, plan.LB, plan.sched)) e = nullptr;
    }
    if (!e && form == FPCG_LAUNCH_SLAB && !extras_fused_only) {
        e = find_slab(plan.KP, plan.FMT, plan.LB, io_c64 ? 1 : 0);
        if (!entry_takes(e, plan.LB, plan.sched)) e = nullptr;
    }
    if (!e) {
        e = find_entry(plan.KP, plan.FMT, plan.LB, io_c64 ? 1 : 0);
        if (!entry_takes(e, plan.LB, plan.sched)) e = nullptr;
    }
    if (!e && !extras_fused_only) {                   // shapes built only as slab kernels
        e = find_slab(plan.KP, plan.FMT, plan.LB, io_c64 ? 1 : 0);
        if (!entry_takes(e, plan.LB, plan.sched)) e = nullptr;
    }
    if (!e) return fail(FPCG_E_UNSUPPORTED, "no kernel built for this launch (K=%d, format %d, L=%d%s)", K, plan.FMT,
                        plan.LB, extras_fused_only ? ", gain or Gram output" : "");
    const bool indexed = ex && ex->chan_idx;
    const int64_t n = indexed ? ex->n : B;           // workgroups along x
    if (B == 0 || n == 0) return FPCG_OK;
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        for (const auto& t : table())
            for (int sp = 0; sp < 2; ++sp)
                for (int r = 0; r < 2; ++r)
                    if (t.fn[sp][r] && t.lds(sp != 0, r != 0, 1) > 65536)   // the largest layout of that build
                        (void)hipFuncSetAttribute(t.fn[sp][r], hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)t.lds(sp != 0, r != 0, 1));
    });
    if (flags && R > 16) {   // several workgroups per channel OR their flags together
        if (indexed)
            hipLaunchKernelGGL(zero_u32_at, dim3(grid_for(n, 256)), dim3(256), 0, stream, flags, ex->chan_idx, n, B);
        else
            hipLaunchKernelGGL(zero_u32, dim3(grid_for(B, 256)), dim3(256), 0, stream, flags, B);
    }
    FusedParams p;
    p.H = H; p.Y = Y; p.sigma2 = sigma2; p.xhat = xhat; p.labels = labels; p.flags = flags;
    p.B = B; p.Nbs = Nbs; p.K = K; p.R = R; p.qam = qam; p.iters = iters;
    p.refresh_every = plan.sched.refresh_every;
    p.refine_steps = plan.sched.refine_steps;
    p.variant = plan.sched.variant;
    p.m = (int)std::lround(std::sqrt((double)qam));
    p.bits = 0;
    while ((1 << p.bits) < p.m) ++p.bits;
    p.nu = std::sqrt(2.0 * (qam - 1) / 3.0);
    p.chan_idx = indexed ? ex->chan_idx : nullptr;
    p.ab_hist = ex ? ex->ab_hist : nullptr;
    p.gain = ex ? ex->gain : nullptr;
    p.gram_out = ex ? ex->gram_out : nullptr;
    p.mf_out = ex ? ex->mf_out : nullptr;
    p.T_out = ex ? ex->T_out : nullptr;
    p.T_in = ex ? ex->T_in : nullptr;
    const int ncb = (R + 15) / 16;
    if (e->kind == 1) {
        dim3 grid((unsigned)n, (unsigned)((R + 15) / 16));
        const int rf = plan.sched.refresh_every > 0 ? 1 : 0;
        const size_t lds = e->lds(sp != 0, false, plan.sched.refresh_every);
        e->launch[sp][rf](p, grid, lds, stream);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return fail(FPCG_E_DEVICE, "slab kernel launch: %s", hipGetErrorString(err));
        return FPCG_OK;
    }
    if (!ref && !ex && e->pipe_fn[sp] && form == FPCG_LAUNCH_PIPELINED) {
        // pipelined form: persistent two-wave workgroups, as many as fit at once
        const size_t lds = e->pipe_lds(sp != 0, p.refresh_every);
        const int per_cu = pipe_occupancy(ctx->device, e->pipe_fn[sp], lds);
        if (per_cu > 0) {
            const int64_t items = B * ncb;
            const int64_t g = std::min<int64_t>(items, (int64_t)per_cu * cu_count(ctx->device));
            e->pipe_launch[sp](p, dim3((unsigned)g), lds, stream);
            hipError_t err = hipGetLastError();
            if (err != hipSuccess) return fail(FPCG_E_DEVICE, "pipelined kernel launch: %s", hipGetErrorString(err));
            return FPCG_OK;
        }
    }
    dim3 grid((unsigned)n, (unsigned)ncb);
    const size_t lds = e->lds(sp != 0, ref != 0, p.refresh_every);   // within 160 KiB (check_args)
    e->launch[sp][ref](p, grid, lds, stream);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(FPCG_E_DEVICE, "fused kernel launch: %s", hipGetErrorString(err));
    return FPCG_OK;
}

fpcg_status launch_detect(const fpcg_ctx* ctx, hipStream_t stream, const Plan& plan, int64_t B, int32_t Nbs,
                          int32_t K, int32_t R, const void* H, const void* Y, int32_t io_c64, const double* sigma2,
                          int32_t qam, int32_t iters, void* xhat, uint8_t* labels, uint32_t* flags) {
    int form = ctx->launch_form;
    if (form == FPCG_LAUNCH_AUTO) {
        auto it = ctx->tuned.find(tune_key(plan, R, io_c64));
        form = it != ctx->tuned.end() ? it->second : FPCG_LAUNCH_FUSED;
    }
    return launch_detect_form(ctx, stream, plan, form, B, Nbs, K, R, H, Y, io_c64, sigma2, qam, iters, xhat, labels,
                              flags);
}

// ------------------------------------------------------------------ slicer / rounding kernels
template <typename T>
__global__ void slice_kernel(int64_t n, const T* x, int m, int bits, double nu_d, uint8_t* labels) {
    const T nu = (T)nu_d, mm = (T)m;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        labels[i] = slice_label<T>(x[2 * i], x[2 * i + 1], nu, mm, m, bits);
}

__global__ void round_kernel(int64_t n, const float* in, int fmt, float scale, float inv, float* out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = round_to(in[i] * scale, fmt) * inv;
}

}  // namespace fpcg

using namespace fpcg;

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* fpcg_strerror(int32_t status) {
    switch (status) {
        case FPCG_OK: return "ok";
        case FPCG_E_INVAL: return "invalid argument";
        case FPCG_E_NOMEM: return "device memory budget exceeded";
        case FPCG_E_DEVICE: return "HIP runtime error";
        case FPCG_E_UNSUPPORTED: return "configuration not built";
        case FPCG_E_BUSY: return "queue full";
        default: return "unknown status";
    }
}

const char* fpcg_last_error(void) { return g_last_error.c_str(); }

fpcg_status fpcg_create(int32_t device, size_t hbm_budget, const char* tune_table, fpcg_ctx** out) {
    clear_error();
    if (!out) return fail(FPCG_E_INVAL, "out is NULL");
    *out = nullptr;
    if (tune_table) {                                 // validated before any device call
        fpcg_ctx probe;
        fpcg_status st = parse_tune_table(tune_table, &probe);
        if (st != FPCG_OK) return st;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return fail(FPCG_E_DEVICE, "no HIP device");
    if (device < 0 || device >= count) return fail(FPCG_E_INVAL, "device %d not in [0, %d)", device, count);
    ScopedDevice sd(device);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(FPCG_E_DEVICE, "hipMemGetInfo failed");
    {
        fpcg_status st = bind_scratch(device);        // this device is current (ScopedDevice)
        if (st != FPCG_OK) return st;
    }
    fpcg_ctx* c = new fpcg_ctx();
    c->device = device;
    c->budget = hbm_budget ? hbm_budget : (size_t)(0.8 * (double)free_b);
    // the coefficient record of fpcg_detect_ex comes from the device's default
    // stream-ordered pool: keep freed blocks there for the next call instead of
    // returning them to the driver at every synchronisation
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)table();
    if (tune_table) (void)parse_tune_table(tune_table, c);
    *out = c;
    return FPCG_OK;
}

void fpcg_destroy(fpcg_ctx* ctx) { delete ctx; }

fpcg_status fpcg_set_launch_form(fpcg_ctx* ctx, int32_t form) {
    clear_error();
    if (!ctx) return fail(FPCG_E_INVAL, "ctx is NULL");
    const int base = form & ((1 << FPCG_LAUNCH_WAVES_SHIFT) - 1), nw = form >> FPCG_LAUNCH_WAVES_SHIFT;
    if (form < 0 || base > FPCG_LAUNCH_SLAB || !(nw == 0 || nw == 1 || nw == 2 || nw == 4) ||
        (nw && base != FPCG_LAUNCH_FUSED))
        return fail(FPCG_E_INVAL, "launch form %d out of range", form);
    ctx->launch_form = form;
    return FPCG_OK;
}

fpcg_status fpcg_check(int64_t B, int32_t Nbs, int32_t K, int32_t R, int32_t qam_order, int32_t iters,
                       int32_t block_L, const fpcg_schedule* sched) {
    clear_error();
    return check_args(B, Nbs, K, R, qam_order, iters, block_L, sched, nullptr);
}

fpcg_status fpcg_detect(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R, const void* H,
                        const void* Y, int32_t io_c64, const double* sigma2, int32_t qam_order, int32_t iters,
                        int32_t block_L, const fpcg_schedule* sched, void* xhat, uint8_t* labels, uint32_t* flags) {
    clear_error();
    if (!ctx) return fail(FPCG_E_INVAL, "ctx is NULL");
    fpcg_schedule rs;
    fpcg_status st = resolve_schedule(ctx, B, Nbs, K, R, qam_order, iters, block_L, sched, &rs);
    if (st != FPCG_OK) return st;
    Plan plan;
    st = check_args(B, Nbs, K, R, qam_order, iters, block_L, &rs, &plan);
    if (st != FPCG_OK) return st;
    if (B > 0 && (!H || !Y || !sigma2 || !xhat || !labels))
        return fail(FPCG_E_INVAL, "H, Y, sigma2, xhat and labels must be non-NULL");
    ScopedDevice sd(ctx->device);
    return launch_detect(ctx, (hipStream_t)stream, plan, B, Nbs, K, R, H, Y, io_c64, sigma2, qam_order, iters,
                         xhat, labels, flags);
}

}  // extern "C"

namespace fpcg {

// fpcg_detect_ex and its variant without allocation: the coefficient record
// of the kappa output comes from the stream-ordered pool, or (use_static) is
// the static array of this GPU
static fpcg_status detect_ex_impl(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R,
                                  const void* H, const void* Y, int32_t io_c64, const double* sigma2,
                                  int32_t qam_order, int32_t iters, int32_t block_L, const fpcg_schedule* sched,
                                  void* xhat, uint8_t* labels, uint32_t* flags, const int32_t* chan_idx,
                                  int64_t n_idx, float* kappa, float* gain, bool use_static) {
    clear_error();
    if (!ctx) return fail(FPCG_E_INVAL, "ctx is NULL");
    fpcg_schedule rs;
    fpcg_status st = resolve_schedule(ctx, B, Nbs, K, R, qam_order, iters, block_L, sched, &rs);
    if (st != FPCG_OK) return st;
    Plan plan;
    st = check_args(B, Nbs, K, R, qam_order, iters, block_L, &rs, &plan);
    if (st != FPCG_OK) return st;
    if (chan_idx && (n_idx < 0 || n_idx > 0x7fffffffLL))
        return fail(FPCG_E_INVAL, "n_idx=%lld out of range [0, 2^31-1]", (long long)n_idx);
    const int64_t n = chan_idx ? n_idx : B;
    if (n > 0 && (!H || !Y || !sigma2 || !xhat || !labels))
        return fail(FPCG_E_INVAL, "H, Y, sigma2, xhat and labels must be non-NULL");
    if (B == 0 || n == 0) return FPCG_OK;
    ScopedDevice sd(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    LaunchExtra ex;
    ex.chan_idx = chan_idx;
    ex.n = n;
    ex.gain = gain;
    const size_t hist_bytes = kappa && iters > 0 ? (size_t)n * std::min(R, KAPPA_COLS) * iters * 2 * sizeof(float) : 0;
    bool pooled = false;
    if (hist_bytes && use_static) {
        // every entry the kappa kernel reads is written by this launch first,
        // so the array needs no clearing between calls
        if (hist_bytes > (size_t)FPCG_STATIC_SCRATCH_BYTES)
            return fail(FPCG_E_INVAL, "coefficient record of %zu bytes exceeds the static workspace of %zu bytes",
                        hist_bytes, (size_t)FPCG_STATIC_SCRATCH_BYTES);
        ex.ab_hist = scratch_of(ctx->device);
        if (!ex.ab_hist) return fail(FPCG_E_DEVICE, "no static workspace bound for device %d", ctx->device);
    } else if (hist_bytes) {
        void* h = nullptr;
        if (hipMallocAsync(&h, hist_bytes, s) != hipSuccess || !h)
            return fail(FPCG_E_NOMEM, "coefficient record of %zu bytes", hist_bytes);
        ex.ab_hist = static_cast<float*>(h);
        pooled = true;
    }
    st = launch_detect_form(ctx, s, plan, FPCG_LAUNCH_FUSED, B, Nbs, K, R, H, Y, io_c64, sigma2, qam_order, iters,
                            xhat, labels, flags, &ex);
    if (st == FPCG_OK && kappa) st = launch_kappa(s, ex.ab_hist, n, R, iters, chan_idx, B, kappa);
    if (pooled) (void)hipFreeAsync(ex.ab_hist, s);
    return st;
}

}  // namespace fpcg

extern "C" {

fpcg_status fpcg_detect_ex(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R, const void* H,
                           const void* Y, int32_t io_c64, const double* sigma2, int32_t qam_order, int32_t iters,
                           int32_t block_L, const fpcg_schedule* sched, void* xhat, uint8_t* labels, uint32_t* flags,
                           const int32_t* chan_idx, int64_t n_idx, float* kappa, float* gain) {
    return detect_ex_impl(ctx, stream, B, Nbs, K, R, H, Y, io_c64, sigma2, qam_order, iters, block_L, sched, xhat,
                          labels, flags, chan_idx, n_idx, kappa, gain, false);
}

fpcg_status fpcg_detect_ex_static(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R,
                                  const void* H, const void* Y, int32_t io_c64, const double* sigma2,
                                  int32_t qam_order, int32_t iters, int32_t block_L, const fpcg_schedule* sched,
                                  void* xhat, uint8_t* labels, uint32_t* flags, const int32_t* chan_idx,
                                  int64_t n_idx, float* kappa, float* gain) {
    return detect_ex_impl(ctx, stream, B, Nbs, K, R, H, Y, io_c64, sigma2, qam_order, iters, block_L, sched, xhat,
                          labels, flags, chan_idx, n_idx, kappa, gain, true);
}

fpcg_status fpcg_detect_pc(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R, const void* H,
                           const void* Y, int32_t io_c64, const double* sigma2, int32_t qam_order, int32_t iters,
                           int32_t block_L, const fpcg_schedule* sched, void* xhat, uint8_t* labels, uint32_t* flags,
                           void* precond, int32_t mode) {
    clear_error();
    if (mode != FPCG_PRECOND_STORE && mode != FPCG_PRECOND_LOAD)
        return fail(FPCG_E_INVAL, "precond mode %d (FPCG_PRECOND_STORE or FPCG_PRECOND_LOAD)", mode);
    if (block_L <= 0) return fail(FPCG_E_INVAL, "a kept preconditioner needs block_L > 0");
    if (!ctx) return fail(FPCG_E_INVAL, "ctx is NULL");
    fpcg_schedule rs;
    fpcg_status st = resolve_schedule(ctx, B, Nbs, K, R, qam_order, iters, block_L, sched, &rs);
    if (st != FPCG_OK) return st;
    Plan plan;
    st = check_args(B, Nbs, K, R, qam_order, iters, block_L, &rs, &plan);
    if (st != FPCG_OK) return st;
    if (B > 0 && (!H || !Y || !sigma2 || !xhat || !labels || !precond))
        return fail(FPCG_E_INVAL, "H, Y, sigma2, xhat, labels and precond must be non-NULL");
    if (B == 0) return FPCG_OK;
    ScopedDevice sd(ctx->device);
    LaunchExtra ex;
    ex.n = B;
    if (mode == FPCG_PRECOND_STORE) ex.T_out = precond;
    else ex.T_in = precond;
    int form = ctx->launch_form;
    if (form == FPCG_LAUNCH_AUTO) {
        auto it = ctx->tuned.find(tune_key(plan, R, io_c64));
        form = it != ctx->tuned.end() ? it->second : FPCG_LAUNCH_FUSED;
    }
    return launch_detect_form(ctx, (hipStream_t)stream, plan, form, B, Nbs, K, R, H, Y, io_c64, sigma2, qam_order,
                              iters, xhat, labels, flags, &ex);
}

fpcg_status fpcg_gram(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R, const void* H,
                      const void* Y, int32_t io_c64, const double* sigma2, const fpcg_schedule* sched, void* A_out,
                      void* B_out, uint32_t* flags) {
    clear_error();
    if (!ctx) return fail(FPCG_E_INVAL, "ctx is NULL");
    if (!sched) return fail(FPCG_E_INVAL, "sched is NULL");
    fpcg_schedule s = *sched;
    s.refresh_every = 0;
    s.refine_steps = 0;
    s.variant = 0;
    Plan plan;
    fpcg_status st = check_args(B, Nbs, K, R, 4, 0, 0, &s, &plan);
    if (st != FPCG_OK) return st;
    if (B > 0 && (!H || !Y || !sigma2 || !A_out || !B_out))
        return fail(FPCG_E_INVAL, "H, Y, sigma2, A_out and B_out must be non-NULL");
    if (B == 0) return FPCG_OK;
    ScopedDevice sd(ctx->device);
    LaunchExtra ex;
    ex.gram_out = A_out;
    ex.mf_out = B_out;
    return launch_detect_form(ctx, (hipStream_t)stream, plan, FPCG_LAUNCH_FUSED, B, Nbs, K, R, H, Y, io_c64, sigma2, 4,
                              0, nullptr, nullptr, flags, &ex);
}

fpcg_status fpcg_slice(void* stream, int64_t n, const void* x, int32_t x_c64, int32_t qam_order, uint8_t* labels) {
    clear_error();
    if (n < 0) return fail(FPCG_E_INVAL, "n=%lld < 0", (long long)n);
    if (!(qam_order == 4 || qam_order == 16 || qam_order == 64 || qam_order == 256))
        return fail(FPCG_E_INVAL, "qam_order=%d", qam_order);
    if (n == 0) return FPCG_OK;
    if (!x || !labels) return fail(FPCG_E_INVAL, "NULL pointer");
    const int m = (int)std::lround(std::sqrt((double)qam_order));
    int bits = 0;
    while ((1 << bits) < m) ++bits;
    const double nu = std::sqrt(2.0 * (qam_order - 1) / 3.0);
    hipStream_t s = (hipStream_t)stream;
    if (x_c64)
        hipLaunchKernelGGL(slice_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, (const float*)x, m, bits, nu, labels);
    else
        hipLaunchKernelGGL(slice_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, (const double*)x, m, bits, nu, labels);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(FPCG_E_DEVICE, "slice launch: %s", hipGetErrorString(err));
    return FPCG_OK;
}

fpcg_status fpcg_round(void* stream, int64_t n, const float* in, int32_t fmt, float scale, float* out) {
    clear_error();
    if (n < 0) return fail(FPCG_E_INVAL, "n < 0");
    if (fmt != FPCG_F32 && fmt != FPCG_BF16 && fmt != FPCG_F16 && fmt != FPCG_F8E4M3)
        return fail(FPCG_E_INVAL, "fmt=%d must be F32, BF16, F16 or F8E4M3", fmt);
    int ex = 0;
    if (!(scale > 0.f) || std::frexp(scale, &ex) != 0.5f) return fail(FPCG_E_INVAL, "scale must be a power of two");
    if (n == 0) return FPCG_OK;
    if (!in || !out) return fail(FPCG_E_INVAL, "NULL pointer");
    hipLaunchKernelGGL(round_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, n, in, fmt, scale, 1.0f / scale, out);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(FPCG_E_DEVICE, "round launch: %s", hipGetErrorString(err));
    return FPCG_OK;
}

fpcg_status fpcg_select_precision(int32_t N, double kappa, int32_t allow_fp8, int32_t* fmt, double* u_bound) {
    clear_error();
    if (N < 1 || !(kappa >= 1.0) || !std::isfinite(kappa)) return fail(FPCG_E_INVAL, "need N >= 1 and finite kappa >= 1");
    if (!fmt) return fail(FPCG_E_INVAL, "fmt is NULL");
    const double bound = 1.0 / (std::pow((double)N, 1.5) * std::sqrt(kappa));
    if (u_bound) *u_bound = bound;
    // cheapest first; fp16 before bf16 (same matrix-core rate, 3 more significand bits)
    struct Cand { int fmt; double u; };
    const Cand cands[] = {{FPCG_F8E4M3, std::ldexp(1.0, -4)},
                          {FPCG_F16, std::ldexp(1.0, -11)},
                          {FPCG_BF16, std::ldexp(1.0, -8)},
                          {FPCG_F32, std::ldexp(1.0, -24)},
                          {FPCG_F64, std::ldexp(1.0, -53)}};
    for (const Cand& c : cands) {
        if (c.fmt == FPCG_F8E4M3 && !allow_fp8) continue;
        if (c.u < bound) { *fmt = c.fmt; return FPCG_OK; }
    }
    *fmt = FPCG_F64;
    return FPCG_OK;
}

}  // extern "C"
