// Precision policy behind the C ABI: the schedule a NULL schedule stands for
// (eq. heuristic / eq. heuristic_bj with the expected condition number the
// context holds, as the heuristic's footnote allows), the device estimate of
// that expectation (fpcg_expected_kappa), and the context's table of tuned
// launch forms and expectations in a small JSON form (fpcg_create,
// fpcg_tune_table).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "fpcg.h"
#include "fpcg_host.hpp"

namespace fpcg {

// ------------------------------------------------------------------ NULL schedule
fpcg_status resolve_schedule(const fpcg_ctx* ctx, int64_t B, int32_t Nbs, int32_t K, int32_t R, int32_t qam,
                             int32_t iters, int32_t L, const fpcg_schedule* s, fpcg_schedule* out) {
    if (s) {
        *out = *s;
        return FPCG_OK;
    }
    auto it = ctx->kappa.find(fpcg_kappa_key(Nbs, K, L));
    if (it == ctx->kappa.end())
        return fail(FPCG_E_INVAL,
                    "no expected condition number for Nbs=%d K=%d L=%d in the context: pass a schedule, or call "
                    "fpcg_expected_kappa / fpcg_set_kappa first", Nbs, K, L);
    int32_t fmt = FPCG_F64;
    double ub = 0;
    fpcg_status st = fpcg_select_precision(K, it->second, 1, &fmt, &ub);
    if (st != FPCG_OK) return st;
    // the heuristic's format, else the next more precise one built for this
    // shape (a more precise format meets the same bound)
    static const int32_t up[] = {FPCG_F8E4M3, FPCG_F16, FPCG_F32, FPCG_F64};
    int start = 0;
    while (start < 4 && up[start] != fmt) ++start;
    if (start == 4) start = fmt == FPCG_BF16 ? 2 : 3;   // bf16: its next more precise format is fp32
    for (int i = start; i < 4; ++i) {
        const int32_t f = up[i];
        const int32_t w = f == FPCG_F64 ? FPCG_F64 : FPCG_F32;
        fpcg_schedule c = {f, f, w, w, 0, 0, L > 0 ? 2 : 0};
        if (check_args(B, Nbs, K, R, qam, iters, L, &c, nullptr) == FPCG_OK) {
            clear_error();
            *out = c;
            return FPCG_OK;
        }
    }
    return fail(FPCG_E_UNSUPPORTED, "no built schedule for Nbs=%d K=%d L=%d", Nbs, K, L);
}

// ------------------------------------------------------------------ tune table (JSON)
// {"version": 1,
//  "forms": [{"KP": 64, "fmt": 3, "L": 4, "split": 1, "refresh": 1, "c64": 1, "multi": 0, "form": 1025}, ...],
//  "kappa": [{"Nbs": 256, "K": 64, "L": 4, "kappa": 37.9}, ...]}
// Objects of the two arrays hold numbers only; unknown keys are ignored.
namespace {

struct Scan {
    const char* p;
    void ws() { while (*p && std::isspace((unsigned char)*p)) ++p; }
    bool eat(char c) {
        ws();
        if (*p == c) { ++p; return true; }
        return false;
    }
    bool str(std::string& out) {
        ws();
        if (*p != '"') return false;
        const char* q = ++p;
        while (*p && *p != '"') ++p;
        if (*p != '"') return false;
        out.assign(q, p - q);
        ++p;
        return true;
    }
    bool num(double& v) {
        ws();
        char* e = nullptr;
        v = std::strtod(p, &e);
        if (e == p) return false;
        p = e;
        return true;
    }
    // skip one JSON value of any kind (for keys this table does not use)
    bool skip() {
        ws();
        if (*p == '"') { std::string s; return str(s); }
        if (*p == '{' || *p == '[') {
            const char open = *p, close = open == '{' ? '}' : ']';
            int depth = 0;
            bool in_str = false;
            for (; *p; ++p) {
                if (in_str) { if (*p == '"') in_str = false; continue; }
                if (*p == '"') in_str = true;
                else if (*p == open) ++depth;
                else if (*p == close && --depth == 0) { ++p; return true; }
            }
            return false;
        }
        double v;
        if (num(v)) return true;
        for (const char* lit : {"true", "false", "null"}) {
            const size_t n = std::strlen(lit);
            if (std::strncmp(p, lit, n) == 0) { p += n; return true; }
        }
        return false;
    }
    // one object of numbers: {"key": number, ...}
    bool object(std::vector<std::pair<std::string, double>>& kv) {
        if (!eat('{')) return false;
        if (eat('}')) return true;
        do {
            std::string k;
            double v;
            if (!str(k) || !eat(':')) return false;
            ws();
            if (*p == '"' || *p == '{' || *p == '[' || *p == 't' || *p == 'f' || *p == 'n') {
                if (!skip()) return false;
                continue;
            }
            if (!num(v)) return false;
            kv.emplace_back(k, v);
        } while (eat(','));
        return eat('}');
    }
};

bool get(const std::vector<std::pair<std::string, double>>& kv, const char* k, double& v) {
    for (const auto& e : kv)
        if (e.first == k) { v = e.second; return true; }
    return false;
}

bool integral(double v) { return std::isfinite(v) && v == std::floor(v) && std::fabs(v) < 2147483648.0; }

}  // namespace

fpcg_status parse_tune_table(const char* text, fpcg_ctx* ctx) {
    Scan sc{text};
    if (!sc.eat('{')) return fail(FPCG_E_INVAL, "tune table: expected a JSON object");
    std::map<fpcg_tune_key, int> forms;
    std::map<fpcg_kappa_key, double> kap;
    if (!sc.eat('}')) {
        do {
            std::string key;
            if (!sc.str(key) || !sc.eat(':')) return fail(FPCG_E_INVAL, "tune table: expected \"key\": value");
            if (key != "forms" && key != "kappa") {
                if (!sc.skip()) return fail(FPCG_E_INVAL, "tune table: bad value of \"%s\"", key.c_str());
                continue;
            }
            if (!sc.eat('[')) return fail(FPCG_E_INVAL, "tune table: \"%s\" must be an array", key.c_str());
            if (sc.eat(']')) continue;
            do {
                std::vector<std::pair<std::string, double>> kv;
                if (!sc.object(kv)) return fail(FPCG_E_INVAL, "tune table: bad object in \"%s\"", key.c_str());
                if (key == "forms") {
                    double v[8];
                    const char* names[8] = {"KP", "fmt", "L", "split", "refresh", "c64", "multi", "form"};
                    for (int i = 0; i < 8; ++i)
                        if (!get(kv, names[i], v[i]) || !integral(v[i]))
                            return fail(FPCG_E_INVAL, "tune table: a \"forms\" entry needs an integer \"%s\"", names[i]);
                    const int form = (int)v[7];
                    const int base = form & ((1 << FPCG_LAUNCH_WAVES_SHIFT) - 1), nw = form >> FPCG_LAUNCH_WAVES_SHIFT;
                    if (form < 0 || base < FPCG_LAUNCH_FUSED || base > FPCG_LAUNCH_SLAB ||
                        !(nw == 0 || nw == 1 || nw == 2 || nw == 4))
                        return fail(FPCG_E_INVAL, "tune table: launch form %d out of range", form);
                    forms[fpcg_tune_key((int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5], (int)v[6])] = form;
                } else {
                    double nbs, k, l, kv_;
                    if (!get(kv, "Nbs", nbs) || !get(kv, "K", k) || !get(kv, "L", l) || !get(kv, "kappa", kv_) ||
                        !integral(nbs) || !integral(k) || !integral(l))
                        return fail(FPCG_E_INVAL, "tune table: a \"kappa\" entry needs integers Nbs, K, L and a number kappa");
                    if (!(kv_ >= 1.0) || !std::isfinite(kv_))
                        return fail(FPCG_E_INVAL, "tune table: kappa %g must be finite and >= 1", kv_);
                    kap[fpcg_kappa_key((int)nbs, (int)k, (int)l)] = kv_;
                }
            } while (sc.eat(','));
            if (!sc.eat(']')) return fail(FPCG_E_INVAL, "tune table: unterminated \"%s\"", key.c_str());
        } while (sc.eat(','));
        if (!sc.eat('}')) return fail(FPCG_E_INVAL, "tune table: unterminated object");
    }
    sc.ws();
    if (*sc.p) return fail(FPCG_E_INVAL, "tune table: trailing characters");
    for (const auto& e : forms) ctx->tuned[e.first] = e.second;
    for (const auto& e : kap) ctx->kappa[e.first] = e.second;
    return FPCG_OK;
}

}  // namespace fpcg

using namespace fpcg;

extern "C" {

fpcg_status fpcg_tune_table(const fpcg_ctx* ctx, char* buf, size_t cap, size_t* len) {
    clear_error();
    if (!ctx) return fail(FPCG_E_INVAL, "ctx is NULL");
    std::string s = "{\"version\": 1, \"forms\": [";
    char tmp[256];
    bool first = true;
    for (const auto& e : ctx->tuned) {
        std::snprintf(tmp, sizeof tmp,
                      "%s{\"KP\": %d, \"fmt\": %d, \"L\": %d, \"split\": %d, \"refresh\": %d, \"c64\": %d, "
                      "\"multi\": %d, \"form\": %d}",
                      first ? "" : ", ", std::get<0>(e.first), std::get<1>(e.first), std::get<2>(e.first),
                      std::get<3>(e.first), std::get<4>(e.first), std::get<5>(e.first), std::get<6>(e.first), e.second);
        s += tmp;
        first = false;
    }
    s += "], \"kappa\": [";
    first = true;
    for (const auto& e : ctx->kappa) {
        std::snprintf(tmp, sizeof tmp, "%s{\"Nbs\": %d, \"K\": %d, \"L\": %d, \"kappa\": %.17g}", first ? "" : ", ",
                      std::get<0>(e.first), std::get<1>(e.first), std::get<2>(e.first), e.second);
        s += tmp;
        first = false;
    }
    s += "]}";
    if (len) *len = s.size() + 1;
    if (!buf) return FPCG_OK;
    if (cap < s.size() + 1) return fail(FPCG_E_INVAL, "buffer of %zu bytes, %zu needed", cap, s.size() + 1);
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return FPCG_OK;
}

fpcg_status fpcg_set_kappa(fpcg_ctx* ctx, int32_t Nbs, int32_t K, int32_t block_L, double kappa) {
    clear_error();
    if (!ctx) return fail(FPCG_E_INVAL, "ctx is NULL");
    if (Nbs < 1 || K < 1 || block_L < 0) return fail(FPCG_E_INVAL, "Nbs=%d K=%d L=%d", Nbs, K, block_L);
    if (!(kappa >= 1.0) || !std::isfinite(kappa)) return fail(FPCG_E_INVAL, "kappa %g must be finite and >= 1", kappa);
    ctx->kappa[fpcg_kappa_key(Nbs, K, block_L)] = kappa;
    return FPCG_OK;
}

fpcg_status fpcg_expected_kappa(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R,
                                const void* H, const void* Y, int32_t io_c64, const double* sigma2, int32_t block_L,
                                int32_t n_sample, double* kappa) {
    clear_error();
    if (!ctx || !kappa) return fail(FPCG_E_INVAL, "ctx and kappa must be non-NULL");
    if (B < 1 || n_sample < 1) return fail(FPCG_E_INVAL, "B=%lld and n_sample=%d must be >= 1", (long long)B, n_sample);
    if (!H || !Y || !sigma2) return fail(FPCG_E_INVAL, "H, Y and sigma2 must be non-NULL");
    // FP64 iterations over the whole Krylov space the estimate can use; where
    // no FP64 build exists for the class, the most precise built format
    // (symmetric form, else the textbook left form of Alg. 3, whose
    // coefficients are those of the Lanczos process of M_d A)
    const int32_t iters = std::min<int32_t>(K, 32);
    fpcg_schedule f64 = {FPCG_F64, FPCG_F64, FPCG_F64, FPCG_F64, 0, 0, block_L > 0 ? 2 : 0};
    fpcg_status st = check_args(B, Nbs, K, R, 4, iters, block_L, &f64, nullptr);
    if (st == FPCG_E_UNSUPPORTED) {
        static const int32_t fmts[] = {FPCG_F32, FPCG_F16, FPCG_BF16};
        for (int32_t f : fmts) {
            for (int32_t v : {2, 1}) {
                const fpcg_schedule c = {f, f, FPCG_F32, FPCG_F32, 0, 0, block_L > 0 ? v : 0};
                if (check_args(B, Nbs, K, R, 4, iters, block_L, &c, nullptr) == FPCG_OK) {
                    f64 = c;
                    st = FPCG_OK;
                    break;
                }
            }
            if (st == FPCG_OK) break;
        }
        if (st == FPCG_OK) clear_error();
    }
    if (st != FPCG_OK) return st;
    const int64_t n = std::min<int64_t>(n_sample, B);
    const size_t el = io_c64 ? 8 : 16;
    const size_t hb = (size_t)Nbs * K * el, yb = (size_t)Nbs * R * el;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    struct Restore { int d; ~Restore() { if (d >= 0) (void)hipSetDevice(d); } } restore{prev};
    hipStream_t s = (hipStream_t)stream;
    char *dH = nullptr, *dY = nullptr, *dX = nullptr;
    double* dS = nullptr;
    uint8_t* dL = nullptr;
    float* dK = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        for (void* q : {(void*)dH, (void*)dY, (void*)dX, (void*)dS, (void*)dL, (void*)dK})
            if (q) (void)hipFree(q);
    };
    if (hipMalloc((void**)&dH, n * hb) != hipSuccess || hipMalloc((void**)&dY, n * yb) != hipSuccess ||
        hipMalloc((void**)&dX, n * (size_t)K * R * el) != hipSuccess || hipMalloc((void**)&dS, n * 8) != hipSuccess ||
        hipMalloc((void**)&dL, n * (size_t)K * R) != hipSuccess || hipMalloc((void**)&dK, n * 4) != hipSuccess) {
        cleanup();
        return fail(FPCG_E_NOMEM, "expected_kappa: buffers for %lld sampled channels", (long long)n);
    }
    // n channels spread evenly over the batch, gathered into one small batch
    for (int64_t i = 0; i < n; ++i) {
        const int64_t c = (i * B) / n;
        if (hipMemcpyAsync(dH + i * hb, (const char*)H + c * hb, hb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(dY + i * yb, (const char*)Y + c * yb, yb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(dS + i, sigma2 + c, 8, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            cleanup();
            return fail(FPCG_E_DEVICE, "expected_kappa: gathering the sample failed");
        }
    }
    st = fpcg_detect_ex(ctx, stream, n, Nbs, K, R, dH, dY, io_c64, dS, 4, iters, block_L, &f64, dX, dL, nullptr,
                        nullptr, 0, dK, nullptr);
    if (st != FPCG_OK) { cleanup(); return st; }
    std::vector<float> hk((size_t)n);
    if (hipMemcpyAsync(hk.data(), dK, n * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        cleanup();
        return fail(FPCG_E_DEVICE, "expected_kappa: reading the estimates failed");
    }
    cleanup();
    double sum = 0;
    int64_t cnt = 0;
    for (float v : hk)
        if (std::isfinite(v) && v >= 1.f) { sum += v; ++cnt; }
    if (!cnt) return fail(FPCG_E_INVAL, "expected_kappa: no sampled channel gave an estimate");
    *kappa = sum / (double)cnt;
    ctx->kappa[fpcg_kappa_key(Nbs, K, block_L)] = *kappa;
    return FPCG_OK;
}

}  // extern "C"
