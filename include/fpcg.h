/*
 * fpcg.h -- C ABI of the MI355X (gfx950) finite-precision block-Jacobi CG
 * massive-MIMO detector (arXiv 2504.09820).
 *
 * The library computes, for every channel c of a batch and every received
 * vector y_n of that channel,
 *     A = H^H H + sigma^2 I,  b_n = H^H y_n           (Sec. II, eq. inversion)
 *     x_n ~= A^{-1} b_n by I iterations of FP-CG       (Alg. 2) or
 *     of FP-BJ-CG with L x L block-Jacobi blocks       (eq. pre_BJ, Alg. 3)
 * in the precisions of an fpcg_schedule, then slices x_n to square-QAM
 * hard decisions with Gray labels.
 *
 * Conventions shared by every call
 *   - Complex arrays are interleaved (re, im), C order.  io_c64 != 0 means
 *     complex64 (float2) elements, otherwise complex128 (double2).
 *   - H is (B, Nbs, K): H[c][a][k] is the gain from stream k to antenna a.
 *     Y is (B, Nbs, R): R received vectors per channel sharing that H.
 *     xhat is (B, K, R) in the same element type as H and Y; labels is
 *     (B, K, R) uint8; flags is (B) uint32; sigma2 is (B) double.
 *   - sigma2[c] >= 0 is added on the Gram's diagonal (A = H^H H + sigma2 I,
 *     the LMMSE system of eq. inversion); sigma2[c] = 0 gives the
 *     zero-forcing system A = H^H H of the same equation, which is positive
 *     definite only when H has full column rank (K <= Nbs): a singular block
 *     or a breakdown is flagged, never a call error.
 *   - Device pointers are memory of the device the context was created on.
 *     The caller allocates and frees them; the library never frees or keeps
 *     caller memory beyond the asynchronous work it enqueued.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     asynchronously; results are valid once the stream reaches that point.
 *   - Argument errors are returned synchronously, before anything is enqueued.
 *     Numerical outcomes are never call errors: they are reported per channel
 *     through the flag bits below.
 *   - A context may be used by one host thread at a time.
 */
#ifndef FPCG_H
#define FPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FPCG_OK = 0,
    FPCG_E_INVAL = -1,        /* bad argument (null pointer, size, order, L not dividing K, ...) */
    FPCG_E_NOMEM = -2,        /* request does not fit the context's device-memory budget        */
    FPCG_E_DEVICE = -3,       /* a HIP runtime call failed                                      */
    FPCG_E_UNSUPPORTED = -4,  /* valid but not built (e.g. K > 128, schedule combination)       */
    FPCG_E_BUSY = -5          /* serving queue full                                             */
} fpcg_status;

/* Number formats (Table I of the paper, plus OCP fp8 e4m3 "fn"). */
typedef enum {
    FPCG_F64 = 0,
    FPCG_F32 = 1,
    FPCG_BF16 = 2,
    FPCG_F16 = 3,
    FPCG_F8E4M3 = 4
} fpcg_fmt;

/* Per-channel flag bits written to flags[c]. */
enum {
    FPCG_FLAG_NONFINITE = 1,     /* A or b had a non-finite entry; x_hat = 0 for the channel   */
    FPCG_FLAG_BREAKDOWN = 2,     /* phi <= 0 or rho <= 0 (or not finite) froze a column         */
    FPCG_FLAG_BLOCK_NOT_PD = 4,  /* a Jacobi block was not positive definite: diagonal inverse   */
    FPCG_FLAG_FP8_SAT = 8        /* an fp8 operand was not finite after scaling                  */
};

/*
 * Precision schedule.  Alg. 2 and Alg. 3 run the matrix-vector product A p at
 * u_MV, the inner products at u_IP and every other step at u_W.
 *   gram_op : format H and y are rounded to before the Gram / matched filter
 *   mv_op   : u_MV, format of the A and p operands of A p (accumulated in
 *             FP32, or FP64 when mv_op = F64)
 *   ip      : u_IP (must equal work)
 *   work    : u_W: F64 (all-FP64 path) or F32
 *   refresh_every : every k-th iteration replace r by b - A x computed in FP64
 *             on the stored Gram (0 = off)
 *   refine_steps  : FP64 iterative refinement steps: r = H^H (y - H x) -
 *             sigma^2 x in FP64, solve A d = r with the same schedule, x += d
 *   variant : block-Jacobi form (block_L > 0): 0 = Alg. 3 as printed (left
 *             preconditioning, rho = r^H p); 1 = textbook left PCG (rho =
 *             r^H z); 2 = symmetric form (the system of Thm 4): A <- T A T^H,
 *             b <- T b with T = blockdiag(C_i^{-1}), A_i = C_i C_i^H, the
 *             Alg. 2 iteration on it, x = T^H x_bar.  All three give the
 *             same iterates in exact arithmetic; 2 keeps the per-iteration
 *             cost of plain CG.
 * Built combinations: gram_op == mv_op, and work = ip = (mv_op == F64 ? F64 : F32).
 */
typedef struct {
    int32_t gram_op;
    int32_t mv_op;
    int32_t ip;
    int32_t work;
    int32_t refresh_every;
    int32_t refine_steps;
    int32_t variant;
} fpcg_schedule;

typedef struct fpcg_ctx fpcg_ctx;

/* Create a context on HIP device `device`.  `hbm_budget` bounds the device
 * memory the serving queue may hold for in-flight requests (0 = 80 % of the
 * free memory at creation).  `tune_table`: NULL, or a table persisted from
 * fpcg_tune_table (launch forms fpcg_autotune chose per shape class and
 * expected condition numbers per workload class), loaded into the context;
 * FPCG_E_INVAL if it does not parse (checked before any device call).
 * Returns FPCG_E_DEVICE if the device is absent. */
fpcg_status fpcg_create(int32_t device, size_t hbm_budget, const char* tune_table, fpcg_ctx** out);

/* The context's table as NUL-terminated JSON:
 *   {"version": 1,
 *    "forms": [{"KP": .., "fmt": .., "L": .., "split": .., "refresh": .., "c64": .., "multi": .., "form": ..}, ...],
 *    "kappa": [{"Nbs": .., "K": .., "L": .., "kappa": ..}, ...]}
 * (forms: padded K, operand format, block size, symmetric form, refresh on,
 * complex64 I/O, several blocks of received vectors -> the launch form of
 * fpcg_set_launch_form).  *len (may be NULL) receives the bytes needed,
 * terminator included; buf = NULL only queries the length; FPCG_E_INVAL if
 * cap is too small.  Host only. */
fpcg_status fpcg_tune_table(const fpcg_ctx* ctx, char* buf, size_t cap, size_t* len);

/* Expected condition number E{kappa} of the iteration matrix of a workload
 * class (Nbs, K, block_L): A = H^H H + sigma^2 I for block_L = 0, the
 * block-Jacobi preconditioned matrix of eq. heuristic_bj otherwise.  The
 * footnote to eq. heuristic allows the expectation in place of each
 * channel's kappa.  fpcg_set_kappa records a known value;
 * fpcg_expected_kappa estimates it on the device: n_sample channels spread
 * evenly over the batch (H, Y, sigma2 as fpcg_detect, device memory) are
 * gathered and solved with FP64 CG for min(K, 32) steps with the kappa output
 * of fpcg_detect_ex, and *kappa receives the mean of the estimates (a lower
 * estimate of each channel's kappa, exact in exact arithmetic when K <= 32).
 * Where no FP64 build serves (K, block_L) (K = 128 with block_L = 16), the
 * solve runs in the most precise built format (FP32 work; the symmetric form,
 * else the textbook left form of Alg. 3), whose coefficients estimate the
 * same spectrum less accurately.
 * Both record the value in the context for the NULL schedule of
 * fpcg_detect.  fpcg_expected_kappa allocates and frees its own device
 * buffers and synchronises `stream`; FPCG_E_INVAL for bad sizes or NULL
 * pointers, or when no sampled channel gives an estimate. */
fpcg_status fpcg_set_kappa(fpcg_ctx* ctx, int32_t Nbs, int32_t K, int32_t block_L, double kappa);
fpcg_status fpcg_expected_kappa(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R,
                                const void* H, const void* Y, int32_t io_c64, const double* sigma2,
                                int32_t block_L, int32_t n_sample, double* kappa);

/* Waits for the context's own streams, then frees everything it owns. */
void fpcg_destroy(fpcg_ctx* ctx);

/* Launch form of fpcg_detect.
 *   FPCG_LAUNCH_AUTO       (default) the form fpcg_autotune chose for the
 *                          launch's shape class, else the fused form with
 *                          the default waves per channel;
 *   FPCG_LAUNCH_FUSED      one workgroup per channel doing every step;
 *   FPCG_LAUNCH_PIPELINED  (one-wave channels, padded K <= 32, no refinement)
 *                          persistent two-wave workgroups, one wave forming
 *                          the Gram and matched filter of the next channel
 *                          while the other solves the current one from the
 *                          other half of a double buffer in LDS.
 * The fused form may carry a wave count per channel,
 *   FPCG_LAUNCH_FUSED | (nw << FPCG_LAUNCH_WAVES_SHIFT), nw in {1, 2, 4},
 * which runs the workgroup of nw waves where that count is built for the
 * launch's shape class (each wave then holds K/(4 nw) entries of every
 * iterate per lane, so a Jacobi block must fit them), else the default count.
 *   FPCG_LAUNCH_SLAB       (K = 64 and K = 128; no refinement; L = 0 or 4,
 *                          and L = 8 / 16 in the symmetric form)
 *                          K/16 waves per channel, each holding its slab of
 *                          rows of every iterate and its column slab of A in
 *                          registers (the operand copies of A p and of the
 *                          FP64 refresh); for K = 128 with FP64 or FP32
 *                          operands, whose u_W matrix does not fit LDS, the
 *                          only form built.
 * Forms and wave counts run the same per-channel algorithm; the fused and
 * pipelined forms of one wave count are bitwise identical, and other wave
 * counts and the slab form differ in the order in which the products and
 * inner products are summed (another valid rounding order).  A form not
 * built for a launch's shape class falls back to the default.
 * FPCG_E_INVAL for a NULL context or an unknown form. */
enum { FPCG_LAUNCH_AUTO = 0, FPCG_LAUNCH_FUSED = 1, FPCG_LAUNCH_PIPELINED = 2, FPCG_LAUNCH_SLAB = 3 };
#define FPCG_LAUNCH_WAVES_SHIFT 8
fpcg_status fpcg_set_launch_form(fpcg_ctx* ctx, int32_t form);

/* Autotuner: times every launch form (and wave count) built for the shape class of these
 * arguments (padded K, operand format, block size and form, refresh on/off,
 * I/O type, one or several blocks of received vectors) on synthetic inputs
 * of this size, `reps` interleaved launches each (1..1000), and records the
 * fastest in the context for FPCG_LAUNCH_AUTO; *chosen_form (may be NULL)
 * receives it.  Allocates and frees its own device buffers and synchronises
 * `stream`; arguments are validated as by fpcg_detect (B >= 1). */
fpcg_status fpcg_autotune(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R,
                          int32_t io_c64, int32_t qam_order, int32_t iters, int32_t block_L,
                          const fpcg_schedule* sched, int32_t reps, int32_t* chosen_form);

/* Static description of a status code. */
const char* fpcg_strerror(int32_t status);

/* Message of the last failing call on this host thread ("" if none). */
const char* fpcg_last_error(void);

/* Host-only validation of a detect() configuration (no device needed).
 * Returns FPCG_OK, FPCG_E_INVAL or FPCG_E_UNSUPPORTED exactly as
 * fpcg_detect would for the same sizes and schedule (sched = NULL checks the
 * sizes with the all-FP64 schedule). */
fpcg_status fpcg_check(int64_t B, int32_t Nbs, int32_t K, int32_t R, int32_t qam_order,
                       int32_t iters, int32_t block_L, const fpcg_schedule* sched);

/*
 * The detector (Sec. II, Alg. 2 / Alg. 3): Gram and matched filter on the
 * matrix cores, block-Jacobi setup, `iters` (P)CG iterations, optional FP64
 * refresh / refinement, QAM slicer.  One fused kernel; nothing but inputs
 * and outputs touches device memory.
 *   B >= 0 channels (B = 0 is a no-op); Nbs >= 1; 1 <= K <= 128; R >= 1.
 *   One channel's H, Y and x_hat must each stay below 2 GiB at complex128
 *   size (16 Nbs max(K, R) < 2^31, 16 K R < 2^31), else FPCG_E_UNSUPPORTED.
 *   qam_order in {4, 16, 64, 256}; iters >= 0 (0 gives x_hat = 0).
 *   block_L = 0: Alg. 2 (no preconditioner); block_L in {4, 8, 16}: Alg. 3,
 *   block_L must divide K; each lane of the kernel owns whole Jacobi blocks,
 *   so L <= 8 below K = 65 and L = 16 runs the K <= 128 build -- except FP32
 *   operands with L = 16 in the symmetric form (variant 2), built in the
 *   slab form at K <= 64 and K <= 128, where the blocks are the 16 x 16
 *   diagonal tiles.  The slab form at K <= 64 also builds L = 8 in the
 *   symmetric form for fp16, bf16 and FP32 operands (two blocks per tile).
 *   65 <= K <= 128 is built for fp8, fp16 and bf16 operands, left block-Jacobi
 *   forms (variant 0 or 1) and no FP64 refresh (with fp8 also with FP64
 *   refinement), and in the slab form for FP64 and FP32 operands without a
 *   preconditioner and for FP32, fp16 and bf16 operands with L = 16 in the
 *   symmetric form, with or without the FP64 refresh.  Other combinations
 *   return FPCG_E_UNSUPPORTED.
 *   sched = NULL selects the schedule by the precision heuristic (eq.
 *   heuristic for block_L = 0, eq. heuristic_bj otherwise): with kappa the
 *   expected condition number the context holds for (Nbs, K, block_L)
 *   (fpcg_expected_kappa, fpcg_set_kappa, or the tune table of
 *   fpcg_create), the cheapest format whose unit roundoff is below
 *   1 / (K^1.5 sqrt(kappa)) (fpcg_select_precision with fp8 allowed; the next
 *   more precise built format where that one is not built for the shape),
 *   operands of the Gram and of A p in it, u_IP = u_W = FP32 (FP64 for the
 *   FP64 format), no refresh or refinement, the symmetric block-Jacobi form.
 *   FPCG_E_INVAL if the context holds no kappa for that class.
 *   flags may be NULL.
 */
fpcg_status fpcg_detect(fpcg_ctx* ctx, void* stream,
                        int64_t B, int32_t Nbs, int32_t K, int32_t R,
                        const void* H, const void* Y, int32_t io_c64, const double* sigma2,
                        int32_t qam_order, int32_t iters, int32_t block_L,
                        const fpcg_schedule* sched,
                        void* xhat, uint8_t* labels, uint32_t* flags);

/* The detector over a subset of the batch, with an optional per-channel
 * condition-number estimate: the input for choosing each channel's operand
 * format with eq. heuristic / eq. heuristic_bj from its own kappa instead of
 * E{kappa} (the footnote to eq. heuristic allows either).
 *   Arguments B .. flags as fpcg_detect (all arrays cover the whole batch).
 *   chan_idx: NULL, or a device array of n_idx channel indices; only those
 *     channels are detected and only their outputs (xhat, labels, flags,
 *     kappa) are written; indices outside [0, B) are skipped.  n_idx is
 *     ignored when chan_idx is NULL (all B channels).
 *   kappa: NULL, or a device array of B floats: for each detected channel,
 *     the largest over its first min(R, 4) received vectors of
 *     lambda_max(T) / lambda_min(T),
 *     T the Lanczos tridiagonal of the CG coefficients of the first solve
 *     (T[0][0] = 1/alpha_1, T[i][i] = 1/alpha_{i+1} + beta_i/alpha_i,
 *     T[i-1][i]^2 = beta_i/alpha_i^2, from the first min(iters, 32) steps
 *     taken before any breakdown).  It estimates the condition number of
 *     the iteration matrix (A without preconditioner, M_d A or A_bar with
 *     it) from below; NaN when no step was taken (iters = 0, breakdown in
 *     the first step).  Needs a stream-ordered workspace of
 *     n * min(R, 4) * iters * 8 bytes (FPCG_E_NOMEM if it cannot be had).
 *   gain: NULL, or a device array of B * K floats, [channel][user]: for each
 *     detected channel the effective gain of each user's estimate,
 *     mu_k = 1 - sigma^2 (M)_kk, M the block-Jacobi inverse of eq. pre_BJ
 *     (the inverses of A's L x L diagonal blocks, computed in u_W; the
 *     diagonal fallback for a block that is not positive definite) and
 *     diag(A)^{-1} when L = 0.  With L = K it is the exact LMMSE gain
 *     (A^{-1} H^H H)_kk.  The input of fpcg_demap_maxlog.
 *   Always one workgroup per channel (the launch form setting is not used).
 *   Errors as fpcg_detect, plus FPCG_E_INVAL for n_idx outside [0, 2^31). */
fpcg_status fpcg_detect_ex(fpcg_ctx* ctx, void* stream,
                           int64_t B, int32_t Nbs, int32_t K, int32_t R,
                           const void* H, const void* Y, int32_t io_c64, const double* sigma2,
                           int32_t qam_order, int32_t iters, int32_t block_L,
                           const fpcg_schedule* sched,
                           void* xhat, uint8_t* labels, uint32_t* flags,
                           const int32_t* chan_idx, int64_t n_idx, float* kappa, float* gain);

/* fpcg_detect_ex without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The coefficient record of the kappa output lives in
 * a static device array of FPCG_STATIC_SCRATCH_BYTES (16 MiB), one copy per
 * GPU, bound when a context is created on that GPU and held until the process
 * ends; n * min(R, 4) * iters * 8 bytes must fit it (n = n_idx, or B without
 * chan_idx), else FPCG_E_INVAL.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other host threads) race and
 * must be serialised by the caller.  Arguments, results and other errors as
 * fpcg_detect_ex (bitwise the same outputs). */
#define FPCG_STATIC_SCRATCH_BYTES (16u << 20)
fpcg_status fpcg_detect_ex_static(fpcg_ctx* ctx, void* stream,
                                  int64_t B, int32_t Nbs, int32_t K, int32_t R,
                                  const void* H, const void* Y, int32_t io_c64, const double* sigma2,
                                  int32_t qam_order, int32_t iters, int32_t block_L,
                                  const fpcg_schedule* sched,
                                  void* xhat, uint8_t* labels, uint32_t* flags,
                                  const int32_t* chan_idx, int64_t n_idx, float* kappa, float* gain);

/* The block-Jacobi preconditioner (eq. pre_BJ) kept across calls.  As
 * fpcg_detect, with block_L > 0 and `precond` a device array of B * K *
 * block_L complex values in the work precision (complex64 for u_W = FP32,
 * complex128 for FP64), caller-owned: element [b][k][j] is entry (k mod L, j)
 * of T_i = C_i^{-1} for the L-block i holding row k of channel b, C_i C_i^H
 * the i-th diagonal block of that channel's u_W Gram.
 *   mode FPCG_PRECOND_STORE: T is computed as fpcg_detect computes it and
 *     written to `precond` (the results are bitwise those of fpcg_detect);
 *   mode FPCG_PRECOND_LOAD: T is read from `precond` in place of the block
 *     factorisation, and the iteration uses M_d = T^H T (left form) or
 *     T A T^H (symmetric form) of that T: a factor stored for the same
 *     channels (a resident channel set) or for an earlier realisation of
 *     them (a time-varying channel, Sec. V).  No BLOCK_NOT_PD flag then.
 * Channels whose K is padded keep the identity on the padding.  Runs the
 * fused or slab form (FPCG_LAUNCH_PIPELINED runs fused).  FPCG_E_INVAL for
 * block_L = 0, a NULL precond with B > 0, or another mode. */
#define FPCG_PRECOND_STORE 1
#define FPCG_PRECOND_LOAD 2
fpcg_status fpcg_detect_pc(fpcg_ctx* ctx, void* stream,
                           int64_t B, int32_t Nbs, int32_t K, int32_t R,
                           const void* H, const void* Y, int32_t io_c64, const double* sigma2,
                           int32_t qam_order, int32_t iters, int32_t block_L,
                           const fpcg_schedule* sched,
                           void* xhat, uint8_t* labels, uint32_t* flags,
                           void* precond, int32_t mode);

/* Step a0-a1 on its own (Sec. II, eq. inversion): the Gram A = H^H H +
 * sigma^2 I and the matched filter B = H^H Y of every channel, formed exactly
 * as fpcg_detect forms them for `sched` (H and Y rounded to sched->gram_op,
 * per-channel / per-column power-of-two scales for fp8, products accumulated
 * on the matrix cores, sigma^2 added to the rounded diagonal), written in u_W:
 * A_out (B, K, K) and B_out (B, K, R), interleaved complex64 for u_W = F32,
 * complex128 for F64, device memory.  The upper triangle of 16 x 16 tiles is
 * formed and the tiles below it are written as conjugate transposes; inside
 * the diagonal tiles both halves are the matrix cores' own sums, so A is
 * Hermitian up to the FP32 (FP64) rounding of two accumulation orders.
 * flags (may be NULL)
 * receives the flags of this step (NONFINITE, FP8_SAT).  refresh, refinement
 * and variant of `sched` are ignored.  Errors as fpcg_detect; sched must not
 * be NULL. */
fpcg_status fpcg_gram(fpcg_ctx* ctx, void* stream, int64_t B, int32_t Nbs, int32_t K, int32_t R,
                      const void* H, const void* Y, int32_t io_c64, const double* sigma2,
                      const fpcg_schedule* sched, void* A_out, void* B_out, uint32_t* flags);

/* Soft output for a channel decoder (Sec. V evaluates the detector in a coded
 * link, Fig. coding): max-log LLRs of each estimated symbol.  The model of
 * the LMMSE estimate with unit-energy symbols is x_hat = mu s + e, e of
 * variance nu^2 = mu (1 - mu); for each label bit
 *   LLR = (min_{s: bit = 1} |x_hat - mu s|^2 - min_{s: bit = 0} |x_hat - mu s|^2) / nu^2,
 * positive when the bit is more likely 0, over the unit-energy Gray square
 * QAM of fpcg_slice.  mu is clamped to [0, 1]; where nu^2 = 0 (mu = 0: no
 * signal; mu = 1: zero-forcing) an LLR is 0 where the distances tie and
 * +-infinity otherwise; NaN in mu, or NaN or infinity in either component
 * of x, makes all of that symbol's LLRs NaN.
 *   n >= 0 symbols x: complex64 (x_c64 != 0, computed in FP32) or complex128
 *     (computed in FP64), device.
 *   gain: device floats, symbol i uses gain[i / R] (R >= 1): the detector's
 *     [channel][user] gains with x_hat laid out (B, K, R).
 *   llr: device, 16-byte aligned, n * log2(Q) floats, [symbol][bit] with
 *     the label's most significant bit first (the I axis's bits, then Q's).
 *   Asynchronous on `stream`; FPCG_E_INVAL for bad sizes, Q, NULL pointers
 *   or alignment. */
fpcg_status fpcg_demap_maxlog(void* stream, int64_t n, int32_t R, const void* x, int32_t x_c64,
                              const float* gain, int32_t qam_order, float* llr);

/* The same LLRs as 8-bit integers, the input width of common decoders:
 * llr[i][b] = clamp(rint(LLR * scale), -127, 127) with the float LLR of
 * fpcg_demap_maxlog, its product with scale rounded to FP32 and then to the
 * nearest integer (ties to even); a NaN LLR becomes 0.  scale: finite, > 0
 * (e.g. 127 / the largest LLR magnitude the decoder should resolve).
 * llr: device, 8-byte aligned, n * log2(Q) bytes, same order as the float
 * form.  Errors as fpcg_demap_maxlog, plus FPCG_E_INVAL for a bad scale. */
fpcg_status fpcg_demap_maxlog_i8(void* stream, int64_t n, int32_t R, const void* x, int32_t x_c64,
                                 const float* gain, int32_t qam_order, float scale, int8_t* llr);

/* QAM slicer on its own (the detector's epilogue): nearest unit-energy
 * square-QAM point per complex value, decided in FP32 (x_c64 != 0) or FP64.
 * Per axis j = clamp(floor((v nu + m) / 2), 0, m - 1), nu = sqrt(2 (Q-1) / 3),
 * label = (gray(j_I) << log2 m) | gray(j_Q).  n >= 0 values, device pointers. */
fpcg_status fpcg_slice(void* stream, int64_t n, const void* x, int32_t x_c64,
                       int32_t qam_order, uint8_t* labels);

/* Operand rounding used by the detector (the fl(.) operator of Def. 1):
 * out[i] = fmt(in[i] * scale) / scale with round-to-nearest-even, for fmt in
 * {F32, BF16, F16, F8E4M3}; `scale` must be a power of two.  n >= 0 floats,
 * device pointers (in-place allowed). */
fpcg_status fpcg_round(void* stream, int64_t n, const float* in, int32_t fmt, float scale, float* out);

/* Precision heuristic (eq. heuristic / eq. heuristic_bj): u_bound =
 * 1 / (N^1.5 sqrt(kappa)); *fmt = the cheapest format whose unit roundoff is
 * below it (fp8 only if allow_fp8; fp16 preferred over bf16).  Host only. */
fpcg_status fpcg_select_precision(int32_t N, double kappa, int32_t allow_fp8,
                                  int32_t* fmt, double* u_bound);

/* ------------------------------------------------------------------ serving
 * A continuous-batching request loop.  Requests carry host buffers; the
 * server admits a request when its device footprint fits the context's
 * budget and a stream slot is free, copies it in, runs fpcg_detect on that
 * slot's stream and copies the results back.  Requests that arrive while
 * others run are admitted as memory and slots free up, so their work overlaps
 * on the device.  Every channel is computed by its own workgroup in a fixed
 * order, so a request's result is bitwise the same alone and in any mix.
 * The host copies between the request's buffers and pinned staging run on
 * the server's own worker threads; fpcg_poll only schedules. */
typedef struct {
    int64_t B;
    int32_t Nbs, K, R;
    int32_t io_c64;
    int32_t qam_order, iters, block_L;
    fpcg_schedule sched;
    const void* H;        /* host (ignored when `channels` is set) */
    const void* Y;        /* host */
    const double* sigma2; /* host (ignored when `channels` is set) */
    void* xhat;           /* host, written on completion */
    uint8_t* labels;      /* host, written on completion */
    uint32_t* flags;      /* host, written on completion (may be NULL) */
    uint64_t channels;    /* 0, or a channel set from fpcg_server_channels whose
                             B, Nbs, K and io_c64 match: H and sigma^2 are then
                             read from device memory, only Y travels */
} fpcg_request;

typedef struct fpcg_server fpcg_server;

/* Device-resident channel set: H (B, Nbs, K) and sigma2 (B) are copied to the
 * device once (counted against the context's budget) and stay there until
 * released, so that requests for the same channels (further received
 * vectors within a coherence block) carry only Y.  Host buffers may be freed
 * on return.  FPCG_E_NOMEM if the set does not fit next to what the server
 * holds; FPCG_E_INVAL for bad sizes or NULL pointers. */
fpcg_status fpcg_server_channels(fpcg_server* srv, int64_t B, int32_t Nbs, int32_t K, int32_t io_c64,
                                 const void* H, const double* sigma2, uint64_t* handle);

/* Releases a channel set once no queued or running request uses it
 * (FPCG_E_BUSY otherwise; FPCG_E_INVAL for an unknown handle). */
fpcg_status fpcg_server_release(fpcg_server* srv, uint64_t handle);

/* A resident channel set also keeps the block-Jacobi factor T of eq. pre_BJ
 * (as fpcg_detect_pc stores it) for each (block_L, sched.gram_op,
 * sched.work) it is served with, counted against the budget: the first
 * request of that class on the set stores it, later ones read it in place of
 * the block factorisation (bitwise the same results while the channels are
 * unchanged; no factor is kept where it would not fit the budget).
 * fpcg_server_channels_update replaces the set's H and sigma2 (same sizes,
 * host buffers) with the channels' next realisation; with keep_precond the
 * kept factors stay and the following requests precondition with the
 * previous realisation's factor (Sec. V, time-varying channel), without it
 * they are dropped.  FPCG_E_BUSY while a request uses the set. */
fpcg_status fpcg_server_channels_update(fpcg_server* srv, uint64_t handle, const void* H, const double* sigma2,
                                        int32_t keep_precond);

/* n_slots concurrent streams (1..16), queue_cap pending requests (>= 1). */
fpcg_status fpcg_server_create(fpcg_ctx* ctx, int32_t n_slots, int32_t queue_cap, fpcg_server** out);

/* Enqueue a request (validated synchronously).  The host buffers must stay
 * valid until fpcg_poll reports completion.  FPCG_E_BUSY if the queue is
 * full, FPCG_E_NOMEM if the request alone exceeds the budget. */
fpcg_status fpcg_submit(fpcg_server* srv, const fpcg_request* req, uint64_t* ticket);

/* Advance the server (admit, launch, retire) and report whether `ticket` is
 * done (1) or not yet (0).  Never blocks. */
fpcg_status fpcg_poll(fpcg_server* srv, uint64_t ticket, int32_t* done);

/* Advance until every submitted request has completed. */
fpcg_status fpcg_drain(fpcg_server* srv);

/* In-flight requests, queued requests, and device bytes the server holds: its
 * slot buffers (kept for reuse between requests) and resident channel sets;
 * never above the budget. */
fpcg_status fpcg_server_stats(fpcg_server* srv, int32_t* in_flight, int32_t* queued, size_t* bytes_held);

/* Drains, then frees the server. */
void fpcg_server_destroy(fpcg_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* FPCG_H */
