// The fused detector kernel for gfx950.
//
// One workgroup of NW waves handles one channel and one block of up to 16
// received vectors (RHS).  Everything between the input read and the output
// write stays on chip:
//
//   1. Gram and matched filter (Sec. II, eq. inversion): A = H^H H + sigma^2 I
//      and B = H^H Y on the matrix cores, split into real planes:
//        Re A = Hr^T Hr + Hi^T Hi,  Im A = Hr^T Hi - Hi^T Hr,
//        Re B = Hr^T Yr + Hi^T Yi,  Im B = Hr^T Yi - Hi^T Yr.
//      Only the upper triangle of 16x16 complex tiles is formed; the lower
//      one is its conjugate transpose.  A and B land in LDS in u_W.
//   2. Block-Jacobi setup (eq. pre_BJ): every L x L diagonal block is
//      Cholesky-factored, A_i = C_i C_i^H, and T_i = C_i^{-1} is formed by
//      forward substitution, one lane per block row/column.  Alg. 3 as
//      printed (left preconditioning) keeps M_i = T_i^H T_i and applies
//      z = M_d r every iteration; its symmetric form (the system of Thm 4)
//      instead rewrites A <- T A T^H and b <- T b once, runs the Alg. 2
//      iteration on it and returns x = T^H x_bar.  On matrix cores the
//      symmetric form keeps the per-iteration cost of plain CG: z = M_d r is
//      fp32 vector work that costs more than the matrix-core product A p.
//   3. (P)CG (Alg. 2 / Alg. 3): r and p live in registers, x in LDS.  Lane
//      (g, n) of wave w owns column n and the SH complex entries
//      (g*NW + w)*SH + e, e < SH, so Jacobi blocks (L | SH) are lane-local.
//      A p runs on the matrix cores with the u_MV operands in registers or
//      LDS (contraction index packed in the lane's own slot order, so the
//      output tile of one iteration is the input operand of the next without
//      any data movement); inner products are lane-local FMA chains reduced
//      over the four lane groups with cross-lane shuffles.
//   4. Optional FP64 residual refresh r = b - A x on the stored Gram, and FP64
//      iterative refinement through H (r = H^H (y - H x) - sigma^2 x).
//   5. QAM slicer epilogue and the x_hat / label stores.
#pragma once

#include <type_traits>

#include "fpcg_device.hpp"

namespace fpcg {

// received-vector columns whose CG coefficients feed the kappa estimate
constexpr int KAPPA_COLS = 4;

struct FusedParams {
    const void* H;
    const void* Y;
    const double* sigma2;
    void* xhat;
    uint8_t* labels;
    uint32_t* flags;
    int64_t B;
    int32_t Nbs, K, R;
    int32_t qam, iters;
    int32_t refresh_every, refine_steps, variant;
    double nu;     // sqrt(2 (Q - 1) / 3)
    int32_t m, bits;
    // optional: the launch's channels as indices into the batch (NULL: all B
    // in order; grid x = their count), and a record of the first solve's CG
    // coefficients of the first min(R, KAPPA_COLS) received-vector columns,
    // [launch position][column][iteration][alpha, beta] (NULL: none)
    const int32_t* chan_idx;
    float* ab_hist;
    // optional: each user's effective gain mu_k = 1 - sigma^2 (M)_kk, M the
    // block-Jacobi inverse of the iteration (diag(A)^{-1} without one),
    // [channel][user] (NULL: none)
    float* gain;
    // optional: the Gram A (K x K) and matched filter B (K x R) of each
    // channel in u_W, interleaved complex, written after step 1; the launch
    // then ends there (no solve, no x_hat or labels; flags of step 1 only)
    void* gram_out;
    void* mf_out;
    // optional: the block-Jacobi factor T = C^{-1} of eq. pre_BJ (C the
    // Cholesky factor of each diagonal block of the u_W Gram), per channel
    // [row k][column j of its L-block] interleaved complex in u_W: written
    // after the setup (T_out), or read in place of the block factorisation
    // (T_in, e.g. the factor of an earlier channel realisation)
    void* T_out;
    const void* T_in;
};

// Lanes of the symmetric block-Jacobi transform.  Pass 1 (rows) needs rows
// m < (b+1) L of block b, pass 2 (columns) columns n >= b L: (b+1) L and
// (NB-b) L items.  A block gets ceil(items / N) lanes for the smallest N
// (items per lane) whose lane total fits the workgroup.
template <int KP, int LB, int NT> struct SplitPlan {
    static constexpr int NB = LB > 0 ? KP / LB : 1;
    static constexpr int items(int b, bool rows) { return (rows ? b + 1 : NB - b) * LB; }
    static constexpr int lanes(int b, bool rows, int n) { return (items(b, rows) + n - 1) / n; }
    static constexpr int total(bool rows, int n) {
        int t = 0;
        for (int b = 0; b < NB; ++b) t += lanes(b, rows, n);
        return t;
    }
    static constexpr int per_lane(bool rows) {
        int n = 1;
        while (total(rows, n) > NT) ++n;
        return n;
    }
    static constexpr int NIR = LB > 0 ? per_lane(true) : 1, NIC = LB > 0 ? per_lane(false) : 1;
    // this lane's block b, its rank r among the block's nl lanes, and whether it serves at all
    __device__ static __forceinline__ void assign(int tid, bool rows, int& b, int& r, int& nl, bool& serves) {
        const int n = rows ? NIR : NIC;
        int first = 0;
        b = 0; r = 0; nl = 1; serves = false;
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            const int c = lanes(bb, rows, n);
            if (tid >= first && tid < first + c) { b = bb; r = tid - first; nl = c; serves = true; }
            first += c;
        }
    }
};

template <int KP_, int NW_, int FMT_, int LB_> struct Cfg {
    static constexpr int KP = KP_, NW = NW_, FMT = FMT_, LB = LB_;
    static constexpr bool LOWP = (FMT != F64 && FMT != F32);
    static constexpr int SH = KP / (4 * NW);          // complex entries per lane group and wave
    static constexpr int NF = SH / 4;                 // 16-row output tiles per wave (Re or Im)
    static constexpr int KPL = LOWP ? (SH % 8 == 0 ? 8 : 4) : 1;
    static constexpr int NKB = SH / KPL;              // contraction blocks per source wave
    static constexpr int F = KP / 16;                 // complex 16-column fragments of H
    static constexpr int KPLG = LOWP ? 8 : 1;         // Gram contraction values per lane and MFMA
    static constexpr int NSUB = LOWP ? 1 : (F <= 2 ? 8 : 4);   // Gram MFMAs per loaded block
    static constexpr int KBG = 4 * KPLG * NSUB;       // antennas per loaded Gram block
    using O = Op<FMT, KPL>;
    using OG = Op<FMT, KPLG>;
    using Wt = typename O::work;
    static constexpr int NAV = NF * NW * NKB * 2;     // u_MV A-operand fragments per lane
    using frag = typename O::frag;
    // A operand: registers when small, else fragment-ordered LDS copy (reduced
    // precision) or read in place from the u_W Gram (fp32 / fp64)
    static constexpr bool AREG = LOWP ? (NAV * (int)sizeof(frag) <= 128) : (NAV * (int)sizeof(Wt) <= 256);
    // K = 128: the u_W Gram does not fit LDS next to everything else, so A is
    // kept only in the operand format, row-major (and its diagonal blocks in
    // u_W for the block-Jacobi setup); built for the reduced formats, left form
    static constexpr bool AROW = KP >= 128;
    static_assert(!AROW || LOWP, "K = 128 keeps A in a reduced operand format");
    static constexpr bool AFRAG_LDS = LOWP && !AREG && !AROW;
    static constexpr size_t ESZ = (FMT == F8) ? 1 : 2;   // bytes of one operand element (AROW)
    static constexpr int NPAIR = F * (F + 1) / 2;
    static constexpr int PPW = (NPAIR + NW - 1) / NW;
    static constexpr int MFPW = (F + NW - 1) / NW;
    static constexpr int LDA = KP + 1;
    static constexpr int RC = NW >= 4 ? 8 : 16;       // antennas per refinement chunk
    static constexpr int NT = 64 * NW;
    // waves per SIMD the register allocation must allow without FP64
    // refinement (1 = no constraint): three for one-wave K <= 32 channels
    static constexpr int MIN_WAVES = (KP <= 32 && FMT != F64) ? 3 : 1;
    // LDS layout in bytes: [Ar | Ai | Br | Bi | M | F | S | X | X64]
    static constexpr size_t W = sizeof(Wt);
    static constexpr size_t sz_Aplane = AROW ? (size_t)KP * KP * ESZ : W * KP * LDA;
    static constexpr size_t off_Ar = 0;
    static constexpr size_t off_Ai = off_Ar + sz_Aplane;
    static constexpr size_t off_Br = off_Ai + sz_Aplane;
    static constexpr size_t off_Bi = off_Br + W * KP * 16;
    static constexpr size_t off_M = off_Bi + W * KP * 16;
    static constexpr size_t sz_M = LB ? 2 * W * KP * LB : 0;           // M_d or T blocks
    static constexpr size_t off_F = off_M + sz_M;                       // A operand fragments
    static constexpr size_t sz_F = AFRAG_LDS ? (size_t)NAV * NT * sizeof(frag) : 0;
    static constexpr size_t off_S = off_F + sz_F;                       // scratch: BJ factors or exchange
    // BJ setup scratch: T = C^{-1} for the left form before M = T^H T (the
    // symmetric form writes T straight into M)
    __host__ __device__ static constexpr size_t sz_bj(bool split) {
        return (LB && !split) ? (LB > 8 ? 4 : 2) * W * KP * LB : 0;   // L = 16 also exchanges C here
    }
    static constexpr size_t sz_xp = (NW > 1) ? (size_t)NW * 64 * 2 * SH * W : 0;    // p exchange (u_W)
    static constexpr size_t sz_red = (NW > 1) ? (size_t)2 * NW * 16 * 4 * W : 0;    // dot partials, 2 parities
    // refinement partials (doubles): used only between two solves, when the
    // p exchange and the dot partials are idle, so they share that region
    static constexpr size_t sz_ref = (NW > 1) ? (size_t)NW * RC * 16 * 2 * 8 : 0;
    static constexpr size_t sz_ex = (sz_xp + sz_red) > sz_ref ? (sz_xp + sz_red) : sz_ref;
    __host__ __device__ static constexpr size_t sz_S(bool split) { return sz_bj(split) > sz_ex ? sz_bj(split) : sz_ex; }
    __host__ __device__ static constexpr size_t off_X(bool split) { return off_S + sz_S(split); }   // x slots [2][SH][NT]
    static constexpr size_t sz_X = 2 * W * SH * NT;
    static constexpr size_t sz_X64 = 2 * 8 * (size_t)SH * NT;           // FP64 iterate [2][SH][NT]
    // AROW: the u_W diagonal blocks live in the x slot until the solve starts
    static_assert(!AROW || sz_X >= 2 * W * KP * (LB ? LB : 1), "diagonal blocks fit the x slot");
    static_assert(AROW || sz_X <= 2 * W * KP * LDA, "x fits the Gram's slot");
    static constexpr size_t sz_B = 2 * W * KP * 16;
    static constexpr bool B_FITS = sz_X + sz_B <= 2 * W * KP * LDA;   // x and B in the Gram's slot
    // Once A's operand copy is packed (into registers, or into its own LDS
    // fragment region) and no FP64 refresh reads the stored Gram, the Gram's
    // LDS is dead and x moves into it.
    __host__ __device__ static constexpr bool x_in_gram(int refresh_every) {
        return (AREG || AFRAG_LDS) && refresh_every == 0;
    }
    // Compact layout (one workgroup per channel, no refinement, x in the Gram's
    // slot): B is carried in registers through the block-Jacobi setup and then
    // stored next to x, so the layout is [A (then x, B) | M | F | S].
    __host__ __device__ static constexpr bool compact(bool refine, int refresh_every) {
        return B_FITS && !refine && x_in_gram(refresh_every);
    }
    // bytes of the general layout [A | B | M | F | S | X | X64]
    __host__ __device__ static constexpr size_t lds_general(bool split, bool refine, int refresh_every) {
        return off_X(split) + (x_in_gram(refresh_every) ? 0 : sz_X) + (refine ? sz_X64 : 0);
    }
    // the outputs of one channel with up to 16 received vectors (x_hat with
    // es bytes per element, then its labels) fit the Gram's slot for staging
    __host__ __device__ static constexpr bool stage_fits(size_t es) {
        return (size_t)KP * 16 * es + 16 + (size_t)KP * 16 <= 2 * sz_Aplane;
    }
    // bytes of a one-workgroup-per-channel launch
    __host__ __device__ static constexpr size_t lds(bool split, bool refine, int refresh_every) {
        return compact(refine, refresh_every) ? off_X(split) - sz_B : lds_general(split, refine, refresh_every);
    }
};

// How a call of detect_channel is used: the whole path by every wave of the
// workgroup (FULL), or one role of the pipelined kernel (one wave each).
enum : int { MODE_FULL = 0, MODE_GRAM = 1, MODE_SOLVE = 2 };

// LDS of one wave ordered against itself (the roles of the pipelined kernel
// synchronise only within their own wave)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One channel (and one block of up to 16 received vectors): the Gram and
// matched filter into the buffer `sbuf` ([Ar | Ai | Br | Bi]), then the
// solve from it using the private regions at `spriv` + the Cfg offsets.
template <int KP, int NW, int FMT, int LB, bool SPLIT, bool REF, typename IOT, int MODE>
__device__ __forceinline__ void detect_channel(const FusedParams& P, const int64_t ch, const int cblk,
                                               unsigned char* sbuf, unsigned char* spriv, uint32_t* sgflag,
                                               const int tid) {
    using C = Cfg<KP, NW, FMT, LB>;
    using O = typename C::O;
    using OG = typename C::OG;
    using Wt = typename C::Wt;
    using frag = typename O::frag;
    using gfrag = typename OG::frag;
    using acc_t = typename O::acc;
    constexpr int SH = C::SH, NF = C::NF, NKB = C::NKB, F = C::F, KPL = C::KPL;
    constexpr int KPLG = C::KPLG, KBG = C::KBG, LDA = C::LDA, PPW = C::PPW, MFPW = C::MFPW;
    constexpr int NT = C::NT;
    static_assert(MODE == MODE_FULL || NW == 1, "pipelined roles are one wave each");

    auto bsync = [&]() {
        if constexpr (MODE == MODE_FULL) __syncthreads();
        else wave_sync();
    };
    const bool x_in_gram = C::x_in_gram(P.refresh_every);
    const bool compact = MODE == MODE_FULL && C::compact(REF, P.refresh_every);
    const size_t shift = compact ? C::sz_B : 0;       // the compact layout has no B slot after A
    Wt* sAr = reinterpret_cast<Wt*>(sbuf + C::off_Ar);
    Wt* sAi = reinterpret_cast<Wt*>(sbuf + C::off_Ai);
    Wt* sBr = reinterpret_cast<Wt*>(compact ? sbuf + C::off_Ar + C::sz_X : sbuf + C::off_Br);
    Wt* sBi = sBr + KP * 16;
    Wt* sMr = reinterpret_cast<Wt*>(spriv + C::off_M - shift);
    Wt* sMi = sMr + KP * (LB ? LB : 1);
    constexpr size_t off_X = C::off_X(LB > 0 && SPLIT);
    Wt* sXr = reinterpret_cast<Wt*>(x_in_gram ? sbuf + C::off_Ar : spriv + off_X);   // x, [SH][NT]
    Wt* sXi = sXr + SH * NT;
    frag* sF = reinterpret_cast<frag*>(spriv + C::off_F - shift);
    double* sX64r = reinterpret_cast<double*>(spriv + off_X + (x_in_gram ? 0 : C::sz_X));   // refinement only
    double* sX64i = sX64r + SH * NT;
    unsigned char* scr = spriv + C::off_S - shift;
    Wt* sXP = reinterpret_cast<Wt*>(scr);                               // [NW][64][2*SH]
    Wt* sRed = reinterpret_cast<Wt*>(scr + C::sz_xp);                  // [2][NW][16][4]
    double* sRef = reinterpret_cast<double*>(scr);                      // [NW][RC][16][2], between solves
    __shared__ uint32_t sFlag;
    __shared__ float sMaxW[NW];
    __shared__ float sMaxC[NW][16];

    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int col = cblk * 16 + n;
    const bool colv = col < P.R;
    const int K = P.K, Nbs = P.Nbs, R = P.R;
    const int64_t hoff = ch * (int64_t)Nbs * K;
    const int64_t yoff = ch * (int64_t)Nbs * R;
    constexpr uint32_t ES = CxB<IOT>::bytes;
    const Buf bH(static_cast<const char*>(P.H) + hoff * ES, (uint32_t)Nbs * K * ES);   // this channel's H
    const Buf bY(static_cast<const char*>(P.Y) + yoff * ES, (uint32_t)Nbs * R * ES);   // this channel's Y
    // this channel's outputs (x_hat, labels) and the per-lane part of their
    // offsets: an invalid received-vector column stores nothing, and padded
    // rows fall past the end of the ranges
    // Outputs.  With one block of received vectors per channel (R <= 16) and
    // a whole-channel workgroup, x_hat and the labels are staged in the
    // Gram's LDS slot (dead once the last solve is done) and written as
    // 16-byte chunks of the channel's contiguous output blocks, x_hat
    // non-temporal: whole lines instead of one 14-element row segment per
    // lane group (measured at c2: less write traffic and shorter launches).
    // Otherwise each element goes straight out through the channel's buffer
    // ranges; padded rows and columns fall outside them and are dropped.
    const bool stage = C::stage_fits(ES) && MODE == MODE_FULL && R <= 16;
    unsigned char* so_x = sbuf + C::off_Ar;
    unsigned char* so_l = so_x + (((size_t)K * R * ES + 15) & ~(size_t)15);
    auto out_begin = [&]() { if (stage) bsync(); };   // every wave is done with the Gram's slot
    auto store_out = [&](int c, auto xr, auto xi, uint8_t label) {
        if (stage) {
            if (colv && c < K) {
                const int o = c * R + col;
                IOT* px = reinterpret_cast<IOT*>(so_x + (size_t)o * ES);
                px[0] = (IOT)xr;
                px[1] = (IOT)xi;
                so_l[o] = label;
            }
        } else {
            const Buf bXo(static_cast<char*>(P.xhat) + (int64_t)ch * K * R * ES, (uint32_t)K * R * ES);
            const Buf bLo(P.labels + (int64_t)ch * K * R, (uint32_t)K * R);
            const uint32_t o = (uint32_t)c * R;
            CxB<IOT>::store(bXo, (colv ? (uint32_t)col * ES : OOB) + o * ES, xr, xi);
            store_u8(bLo, (colv ? (uint32_t)col : OOB) + o, label);
        }
    };
    auto out_end = [&]() {
        if (!stage) return;
        bsync();
        const Buf bXo(static_cast<char*>(P.xhat) + (int64_t)ch * K * R * ES, (uint32_t)K * R * ES);
        const Buf bLo(P.labels + (int64_t)ch * K * R, (uint32_t)K * R);
        const uint32_t nx = (uint32_t)K * R * ES, nl = (uint32_t)K * R;
        for (uint32_t i = tid * 16u; i + 16u <= nx; i += NT * 16u)
            store_b128<CP_STREAM>(bXo, i, *reinterpret_cast<const u32x4v*>(so_x + i));
        if ((nx & 15u) && tid == 0) {                   // an odd element count leaves 8 bytes
            const uint32_t i = nx & ~15u;
            store_b64<CP_STREAM>(bXo, i, *reinterpret_cast<const u32x2v*>(so_x + i));
        }
        for (uint32_t i = tid * 16u; i + 16u <= nl; i += NT * 16u)
            store_b128<0>(bLo, i, *reinterpret_cast<const u32x4v*>(so_l + i));
        for (uint32_t i = (nl & ~15u) + tid; i < nl; i += NT) store_u8(bLo, i, so_l[i]);
    };
    auto hofs = [&](int a, int k) -> uint32_t { return (a < Nbs && k < K) ? ((uint32_t)a * K + k) * ES : OOB; };
    auto yofs = [&](int a) -> uint32_t { return (a < Nbs && colv) ? ((uint32_t)a * R + col) * ES : OOB; };
    const double s2 = P.sigma2[ch];
    if constexpr (MODE == MODE_FULL) {
        if (tid == 0) sFlag = 0u;
    }
    uint32_t myflag = 0u;

    // block-wide max over one float per thread (fixed order, result in all threads)
    auto block_max = [&](float v) -> float {
        v = wave_max(v);
        if constexpr (NW > 1) {
            __syncthreads();
            if (lane == 0) sMaxW[wave] = v;
            __syncthreads();
            v = sMaxW[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) v = fmaxf(v, sMaxW[w]);
        }
        return v;
    };
    // max over the lanes of one column, across waves
    auto column_max = [&](float v) -> float {
        v = col_max(v);
        if constexpr (NW > 1) {
            __syncthreads();
            if (g == 0) sMaxC[wave][n] = v;
            __syncthreads();
            v = sMaxC[0][n];
#pragma unroll
            for (int w = 1; w < NW; ++w) v = fmaxf(v, sMaxC[w][n]);
        }
        return v;
    };

    // B carried in registers (compact layout), stored once A is packed
    Wt bcr[C::MFPW][4], bci[C::MFPW][4];
    int eA = 0;                                       // fp8: exponent of the iteration matrix's scale
    unsigned char* sA8r = sbuf + C::off_Ar;           // AROW: A in the operand format, row-major
    unsigned char* sA8i = sbuf + C::off_Ai;
    Wt* sDr = reinterpret_cast<Wt*>(spriv + C::off_X(false));   // AROW: u_W diagonal blocks (x slot)
    Wt* sDi = sDr + KP * (LB ? LB : 1);
    if constexpr (MODE != MODE_SOLVE) {
    // ------------------------------------------------------------ fp8 scales
    int eH = 0, eY = 0;
    if constexpr (FMT == F8) {
        // eight range-checked loads in flight per lane (out of range reads zero)
        float mh = 0.f;
        const int nh = Nbs * K;
        for (int i0 = 0; i0 < nh; i0 += 8 * NT) {
            float re[8], im[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + u * NT + tid;
                CxB<IOT>::load(bH, i < nh ? (uint32_t)i * ES : OOB, re[u], im[u]);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) mh = fmaxf(mh, fmaxf(fabsf(re[u]), fabsf(im[u])));
        }
        mh = block_max(mh);
        float my = 0.f;
        for (int a0 = g + 4 * wave; a0 < Nbs; a0 += 32 * NW) {
            float re[8], im[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) CxB<IOT>::load(bY, yofs(a0 + u * 4 * NW), re[u], im[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u) my = fmaxf(my, fmaxf(fabsf(re[u]), fabsf(im[u])));
        }
        my = column_max(my);
        eH = fp8_scale_exp(mh);
        eY = fp8_scale_exp(my);
    }
    const float sH = ldexpf(1.f, eH), sY = ldexpf(1.f, eY);

    // ------------------------------------------------------------ 1. Gram + matched filter
    {
        acc_t gAr[PPW], gAi[PPW], gBr[MFPW], gBi[MFPW];
#pragma unroll
        for (int s = 0; s < PPW; ++s) { gAr[s] = acc_t{0, 0, 0, 0}; gAi[s] = acc_t{0, 0, 0, 0}; }
#pragma unroll
        for (int s = 0; s < MFPW; ++s) { gBr[s] = acc_t{0, 0, 0, 0}; gBi[s] = acc_t{0, 0, 0, 0}; }

        constexpr int NSUB = C::NSUB, NLD = KPLG * NSUB;
        // per-lane part of the load offsets, fixed for the whole loop: a padded
        // user column (k >= K) or received-vector column (col >= R) starts at
        // OOB, so every load of it reads zero; antennas a >= Nbs lie past the
        // end of the channel's range and read zero as well
        uint32_t hl[F];
#pragma unroll
        for (int f = 0; f < F; ++f) hl[f] = (16 * f + n < K) ? (uint32_t)(16 * f + n) * ES : OOB;
        const uint32_t yl = colv ? (uint32_t)col * ES : OOB;
        const uint32_t hrow = (uint32_t)K * ES, yrow = (uint32_t)R * ES;
        // H rows that are whole 128-byte lines stream non-temporally (one
        // loop per cache policy: the policy is part of the instruction)
        auto gram_loop = [&](auto hcp) {
            for (int a0 = 0; a0 < Nbs; a0 += KBG) {
                // range-checked loads: all loads of the block in flight together;
                // lane (g, n) takes antennas a0 + g NLD + j, j < NLD, the same for H
                // and Y, so every MFMA contracts matching antennas
                Wt hr[F][NLD], hi[F][NLD], yr[NLD], yi[NLD];
                const uint32_t ab = (uint32_t)(a0 + g * NLD);
#pragma unroll
                for (int j = 0; j < NLD; ++j) {
#pragma unroll
                    for (int f = 0; f < F; ++f) CxB<IOT>::template load<decltype(hcp)::value>(bH, hl[f] + (ab + j) * hrow, hr[f][j], hi[f][j]);
                    CxB<IOT>::load(bY, yl + (ab + j) * yrow, yr[j], yi[j]);
                }
#pragma unroll
                for (int u = 0; u < NSUB; ++u) {
                    gfrag Xr[F], Xi[F], nXi[F];
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        Xr[f] = OG::pack(&hr[f][u * KPLG], sH);
                        Xi[f] = OG::pack(&hi[f][u * KPLG], sH);
                        nXi[f] = OG::neg(Xi[f]);
                    }
                    const gfrag Yr = OG::pack(&yr[u * KPLG], sY), Yi = OG::pack(&yi[u * KPLG], sY);
                    int q = 0;
#pragma unroll
                    for (int f1 = 0; f1 < F; ++f1) {
#pragma unroll
                        for (int f2 = f1; f2 < F; ++f2) {
                            if (NW == 1 || q % NW == wave) {
                                const int s = q / NW;
                                gAr[s] = OG::mfma(Xr[f1], Xr[f2], gAr[s]);
                                gAr[s] = OG::mfma(Xi[f1], Xi[f2], gAr[s]);
                                gAi[s] = OG::mfma(Xr[f1], Xi[f2], gAi[s]);
                                gAi[s] = OG::mfma(nXi[f1], Xr[f2], gAi[s]);
                            }
                            ++q;
                        }
                    }
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        if (NW == 1 || f % NW == wave) {
                            const int s = f / NW;
                            gBr[s] = OG::mfma(Xr[f], Yr, gBr[s]);
                            gBr[s] = OG::mfma(Xi[f], Yi, gBr[s]);
                            gBi[s] = OG::mfma(Xr[f], Yi, gBi[s]);
                            gBi[s] = OG::mfma(nXi[f], Yr, gBi[s]);
                        }
                    }
                }
            }
        };
        if (hrow % 128u == 0) gram_loop(std::integral_constant<int, CP_STREAM>{});
        else gram_loop(std::integral_constant<int, 0>{});

        // scale back (fp8), add sigma^2, mirror into LDS
        const Wt invH = (Wt)ldexpf(1.f, -eH), invY = (Wt)ldexpf(1.f, -eY);
        const Wt s2w = (Wt)s2;
        bool bad = false;
        // non-finite check of many values at one FMA each: v * 0 is NaN exactly
        // when v is infinite or NaN, and a NaN stays in the sum
        Wt nfa = 0;
        // the u_W value of one Gram element (sigma^2 on the diagonal, padding diagonal 1)
        auto gram_at = [&](int s, int jj, int row, int cc, Wt& ar, Wt& ai) {
            ar = (Wt)gAr[s][jj];
            ai = (Wt)gAi[s][jj];
            if constexpr (FMT == F8) { ar = ar * invH * invH; ai = ai * invH * invH; }
            if (row == cc) {
                ai = 0;
                ar = (row < K) ? ar + s2w : (Wt)1;
            }
        };
        if constexpr (C::AROW) {
            // largest magnitude first (fp8 scale), then the operand-format bits of
            // both triangles and the u_W diagonal blocks; padding entries are zero
            // in the operand so that they contribute exactly nothing to A p
            float amax = 0.f;
            int q = 0;
#pragma unroll
            for (int f1 = 0; f1 < F; ++f1)
#pragma unroll
                for (int f2 = f1; f2 < F; ++f2) {
                    if (NW == 1 || q % NW == wave) {
                        const int s = q / NW;
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const int row = 16 * f1 + OG::crow(g, jj), cc = 16 * f2 + n;
                            Wt ar, ai;
                            gram_at(s, jj, row, cc, ar, ai);
                            const bool nf = !__builtin_isfinite(ar) || !__builtin_isfinite(ai);
                            bad |= nf;
                            if constexpr (FMT == F8) {
                                if (nf && row < K && cc < K) myflag |= FLAG_FP8_SAT;
                            }
                            if (row < K && cc < K) amax = fmaxf(amax, fmaxf(fabsf((float)ar), fabsf((float)ai)));
                        }
                    }
                    ++q;
                }
            if constexpr (FMT == F8) eA = fp8_scale_exp(block_max(amax));
            const float sAs = ldexpf(1.f, eA);
            auto put = [&](unsigned char* base, int idx, float v) {
                const uint32_t b = op_bits<FMT>(v);
                if constexpr (C::ESZ == 1) base[idx] = (unsigned char)b;
                else reinterpret_cast<uint16_t*>(base)[idx] = (uint16_t)b;
            };
            q = 0;
#pragma unroll
            for (int f1 = 0; f1 < F; ++f1)
#pragma unroll
                for (int f2 = f1; f2 < F; ++f2) {
                    if (NW == 1 || q % NW == wave) {
                        const int s = q / NW;
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const int row = 16 * f1 + OG::crow(g, jj), cc = 16 * f2 + n;
                            Wt ar, ai;
                            gram_at(s, jj, row, cc, ar, ai);
                            const bool real_entry = row < K && cc < K;
                            if (P.gram_out && real_entry && cblk == 0) {
                                Wt* go = static_cast<Wt*>(P.gram_out) + (size_t)ch * K * K * 2;
                                go[2 * (row * K + cc)] = ar;
                                go[2 * (row * K + cc) + 1] = ai;
                                if (f1 != f2) { go[2 * (cc * K + row)] = ar; go[2 * (cc * K + row) + 1] = -ai; }
                            }
                            const float vr = real_entry ? (float)ar * sAs : 0.f;
                            const float vi = real_entry ? (float)ai * sAs : 0.f;
                            put(sA8r, row * KP + cc, vr);
                            put(sA8i, row * KP + cc, vi);
                            if (f1 != f2) {
                                put(sA8r, cc * KP + row, vr);
                                put(sA8i, cc * KP + row, -vi);
                            }
                            if constexpr (LB > 0) {
                                if (row / LB == cc / LB) {
                                    sDr[row * LB + cc % LB] = ar;
                                    sDi[row * LB + cc % LB] = ai;
                                }
                            } else if constexpr (MODE == MODE_FULL) {
                                // effective gain without a preconditioner: 1 - sigma^2 / a_kk
                                if (P.gain && cblk == 0 && row == cc && row < K)
                                    P.gain[ch * K + row] = (float)((Wt)1 - s2w / ar);
                            }
                        }
                    }
                    ++q;
                }
        } else {
        int q = 0;
#pragma unroll
        for (int f1 = 0; f1 < F; ++f1) {
#pragma unroll
            for (int f2 = f1; f2 < F; ++f2) {
                if (NW == 1 || q % NW == wave) {
                    const int s = q / NW;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int row = 16 * f1 + OG::crow(g, jj), cc = 16 * f2 + n;
                        Wt ar = (Wt)gAr[s][jj], ai = (Wt)gAi[s][jj];
                        if constexpr (FMT == F8) { ar = ar * invH * invH; ai = ai * invH * invH; }
                        if (row == cc) {
                            ai = 0;
                            ar = (row < K) ? ar + s2w : (Wt)1;
                        }
                        nfa = fma(ar, (Wt)0, fma(ai, (Wt)0, nfa));
                        if (P.gram_out && row < K && cc < K && cblk == 0) {
                            Wt* go = static_cast<Wt*>(P.gram_out) + (size_t)ch * K * K * 2;
                            go[2 * (row * K + cc)] = ar;
                            go[2 * (row * K + cc) + 1] = ai;
                            if (f1 != f2) { go[2 * (cc * K + row)] = ar; go[2 * (cc * K + row) + 1] = -ai; }
                        }
                        sAr[row * LDA + cc] = ar;
                        sAi[row * LDA + cc] = ai;
                        if (f1 != f2) {
                            sAr[cc * LDA + row] = ar;
                            sAi[cc * LDA + row] = -ai;
                        }
                    }
                }
                ++q;
            }
        }
        }
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (NW == 1 || f % NW == wave) {
                const int s = f / NW;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int row = 16 * f + OG::crow(g, jj);
                    Wt br = (Wt)gBr[s][jj], bi = (Wt)gBi[s][jj];
                    if constexpr (FMT == F8) { br = br * invH * invY; bi = bi * invH * invY; }
                    nfa = fma(br, (Wt)0, fma(bi, (Wt)0, nfa));
                    if (P.mf_out && row < K && colv) {
                        Wt* mo = static_cast<Wt*>(P.mf_out) + ((size_t)ch * K * R + (size_t)row * R + col) * 2;
                        mo[0] = br;
                        mo[1] = bi;
                    }
                    bcr[s][jj] = br;
                    bci[s][jj] = bi;
                    if (!compact) {
                        sBr[row * 16 + n] = br;
                        sBi[row * 16 + n] = bi;
                    }
                }
            }
        }
        if (bad || !__builtin_isfinite(nfa)) myflag |= FLAG_NONFINITE;
    }
    }
    if constexpr (MODE == MODE_GRAM) {
        // hand the buffer's flag to the solving wave
        const bool nf = __ballot((myflag & FLAG_NONFINITE) != 0) != 0;
        if (tid == 0) *sgflag = nf ? FLAG_NONFINITE : 0u;
        wave_sync();
        return;
    } else {
        if constexpr (MODE == MODE_SOLVE) myflag = *sgflag;
        bsync();
        if constexpr (MODE == MODE_FULL) {
            if (P.gram_out) {                          // step 1 only: its flags, then done
                if (myflag) atomicOr(&sFlag, myflag);
                __syncthreads();
                if (tid == 0 && P.flags) {
                    if (P.R <= 16) P.flags[ch] = sFlag;
                    else if (sFlag) atomicOr(&P.flags[ch], sFlag);
                }
                return;
            }
        }
    }


    constexpr bool split = (LB > 0) && SPLIT;          // symmetric form of Alg. 3
    constexpr bool left = (LB > 0) && !SPLIT;          // Alg. 3 as printed / textbook PCG

    // ------------------------------------------------------------ 2. block-Jacobi setup (eq. pre_BJ)
    if constexpr (LB > 0) {
        Wt* sTr = reinterpret_cast<Wt*>(scr);         // T of the left form (then M = T^H T)
        Wt* sTi = sTr + KP * LB;
        const bool act = tid < KP;
        const int t = act ? tid : 0;
        const int i = t % LB, cb = t - i;             // row in block, first row of block
        // Every lane of a block factors the whole block in registers (the same
        // operations in the same order, so identical results): no exchange.
        // Lower triangle of A_blk; the Cholesky factor C overwrites it, with
        // 1 / c_jj kept in the (otherwise zero) imaginary slot of the diagonal.
        // element (r, c) of this block of the u_W Gram
        auto blk = [&](int r, int c, Wt& re, Wt& im) {
            if constexpr (C::AROW) { re = sDr[(cb + r) * LB + c]; im = sDi[(cb + r) * LB + c]; }
            else { re = sAr[(cb + r) * LDA + cb + c]; im = sAi[(cb + r) * LDA + cb + c]; }
        };
        Wt diag = 0;                                  // a_ii, for the not-PD fallback
        bool blk_bad = false;
        Wt tr[LB], ti[LB];
        // a given factor (T_in, uniform) replaces the factorisation
        const bool factor = MODE != MODE_FULL || !P.T_in;
        if (!factor) {
            if (act && cb < K) {
                const Wt* tin = static_cast<const Wt*>(P.T_in) + ((size_t)ch * K + cb) * LB * 2;
#pragma unroll
                for (int r = 0; r < LB; ++r) { tr[r] = tin[(r * LB + i) * 2]; ti[r] = tin[(r * LB + i) * 2 + 1]; }
            } else {                                  // padding blocks: the identity
#pragma unroll
                for (int r = 0; r < LB; ++r) { tr[r] = r == i ? (Wt)1 : (Wt)0; ti[r] = 0; }
            }
        } else if constexpr (LB <= 8) {
        Wt cr[LB][LB], ci[LB][LB];
#pragma unroll
        for (int r = 0; r < LB; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) blk(r, c, cr[r][c], ci[r][c]);
#pragma unroll
        for (int r = 0; r < LB; ++r)
            if (r == i) diag = cr[r][r];
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            Wt d = cr[j][j];
            if (!(d > 0) || !__builtin_isfinite(d)) { blk_bad = true; d = 1; }
            const Wt l = sqrt(d), inv = (Wt)1 / l;
            cr[j][j] = l;
            ci[j][j] = inv;
#pragma unroll
            for (int r = j + 1; r < LB; ++r) { cr[r][j] = cr[r][j] * inv; ci[r][j] = ci[r][j] * inv; }
#pragma unroll
            for (int r = j + 1; r < LB; ++r)
#pragma unroll
                for (int c = j + 1; c <= r; ++c) {
                    // a_rc -= l_rj conj(l_cj)
                    cr[r][c] = fma(-cr[r][j], cr[c][j], fma(-ci[r][j], ci[c][j], cr[r][c]));
                    ci[r][c] = fma(-ci[r][j], cr[c][j], fma(cr[r][j], ci[c][j], ci[r][c]));
                }
        }
        // T = C^{-1}: this lane forms column i by forward substitution;
        // t_m = 0 for m < i, so full-length sums add exact zeros
#pragma unroll
        for (int r = 0; r < LB; ++r) {
            const Wt inv_rr = ci[r][r];
            Wt sr = 0, si = 0;
#pragma unroll
            for (int m = 0; m < r; ++m) {
                sr = fma(cr[r][m], tr[m], fma(-ci[r][m], ti[m], sr));
                si = fma(cr[r][m], ti[m], fma(ci[r][m], tr[m], si));
            }
            tr[r] = (r == i) ? inv_rr : (r > i ? -sr * inv_rr : (Wt)0);
            ti[r] = (r > i) ? -si * inv_rr : (Wt)0;
        }
        } else {
        // L = 16: a whole block does not fit one lane's registers.  Lane i owns
        // row i of the block; C is exchanged through LDS (the imaginary
        // diagonal slot again holding 1 / c_jj), one column per step.
        Wt* sLr = sTr + 2 * KP * LB;                  // after the T scratch
        Wt* sLi = sLr + KP * LB;
        Wt ar[LB], ai[LB];
#pragma unroll
        for (int c = 0; c < LB; ++c) blk(i, c, ar[c], ai[c]);
#pragma unroll
        for (int c = 0; c < LB; ++c)
            if (c == i) diag = ar[c];
        bool bad = false;
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            if (act && i == j) {
                Wt d = ar[j];
                if (!(d > 0) || !__builtin_isfinite(d)) { bad = true; d = 1; }
                const Wt l = sqrt(d);
                sLr[(cb + j) * LB + j] = l;
                sLi[(cb + j) * LB + j] = (Wt)1 / l;
            }
            bsync();
            const Wt inv = sLi[(cb + j) * LB + j];
            const Wt lr = ar[j] * inv, li = ai[j] * inv;
            if (act && i > j) {
                sLr[(cb + i) * LB + j] = lr;
                sLi[(cb + i) * LB + j] = li;
            }
            bsync();
            if (i > j) {
                Wt kr[LB], ki[LB];
#pragma unroll
                for (int k = j + 1; k < LB; ++k) { kr[k] = sLr[(cb + k) * LB + j]; ki[k] = sLi[(cb + k) * LB + j]; }
#pragma unroll
                for (int k = j + 1; k < LB; ++k) {   // a_ik -= l_ij conj(l_kj), needed for k <= i
                    ar[k] = fma(-lr, kr[k], fma(-li, ki[k], ar[k]));
                    ai[k] = fma(-li, kr[k], fma(lr, ki[k], ai[k]));
                }
            }
        }
        // the block's lanes are one aligned group of LB lanes of a wave
        const uint64_t bal = __ballot(act && bad);
        blk_bad = ((bal >> (lane & ~(LB - 1))) & ((LB == 64) ? ~0ull : ((1ull << LB) - 1))) != 0;
#pragma unroll
        for (int r = 0; r < LB; ++r) {
            const Wt inv_rr = sLi[(cb + r) * LB + r];
            Wt sr = 0, si = 0;
#pragma unroll
            for (int m = 0; m < r; ++m) {
                const Wt cr_ = sLr[(cb + r) * LB + m], ci_ = sLi[(cb + r) * LB + m];
                sr = fma(cr_, tr[m], fma(-ci_, ti[m], sr));
                si = fma(cr_, ti[m], fma(ci_, tr[m], si));
            }
            tr[r] = (r == i) ? inv_rr : (r > i ? -sr * inv_rr : (Wt)0);
            ti[r] = (r > i) ? -si * inv_rr : (Wt)0;
        }
        }
        if (blk_bad) {
            // not positive definite: T = diag(a_ii)^{-1/2}, so M_d = diag(a_ii)^{-1}
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                tr[r] = 0; ti[r] = 0;
                if (r == i) tr[r] = (diag > 0 && __builtin_isfinite(diag)) ? (Wt)1 / sqrt(diag) : (Wt)1;
            }
        }
        Wt* dTr = split ? sMr : sTr;                  // the symmetric form keeps T itself
        Wt* dTi = split ? sMi : sTi;
        if (act) {
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                dTr[(cb + r) * LB + i] = tr[r];
                dTi[(cb + r) * LB + i] = ti[r];
            }
            if constexpr (MODE == MODE_FULL) {
                if (P.T_out && cblk == 0 && cb < K) {  // column i of this block of T
                    Wt* tout = static_cast<Wt*>(P.T_out) + ((size_t)ch * K + cb) * LB * 2;
#pragma unroll
                    for (int r = 0; r < LB; ++r) { tout[(r * LB + i) * 2] = tr[r]; tout[(r * LB + i) * 2 + 1] = ti[r]; }
                }
            }
            if (blk_bad && i == 0) myflag |= FLAG_BLOCK_NOT_PD;
            if constexpr (MODE == MODE_FULL) {
                // (M_d)_ii = sum over the rows of |T[r][i]|^2: column i of T is this lane's
                if (P.gain && cblk == 0 && t < K) {
                    Wt mii = 0;
#pragma unroll
                    for (int r = 0; r < LB; ++r) mii = fma(tr[r], tr[r], fma(ti[r], ti[r], mii));
                    P.gain[ch * K + t] = (float)((Wt)1 - (Wt)s2 * mii);
                }
            }
        }
        bsync();
        if constexpr (!split) {
            // M = T^H T: row i
            // with column i of T in this lane's registers; T is lower triangular
            // with zeros stored above the diagonal, so full-length sums add exact zeros
            if (act) {
#pragma unroll
                for (int j = 0; j < LB; ++j) {
                    Wt mr = 0, mi = 0;
#pragma unroll
                    for (int m = 0; m < LB; ++m) {
                        const Wt br_ = sTr[(cb + m) * LB + j], bi_ = sTi[(cb + m) * LB + j];   // T[m][j]
                        mr = fma(tr[m], br_, fma(ti[m], bi_, mr));                           // conj(T[m][i]) T[m][j]
                        mi = fma(tr[m], bi_, fma(-ti[m], br_, mi));
                    }
                    sMr[(cb + i) * LB + j] = mr;
                    sMi[(cb + i) * LB + j] = mi;
                }
            }
            bsync();
        } else {
            // A <- T A T^H in place, upper triangle only (the lower one is read as
            // its conjugate, the diagonal as real: the result is Hermitian by
            // construction).  T is block lower triangular, so
            //   W = A T^H:   W[m][bL + c] = sum_{j <= c} A[m][bL + j] conj(T[bL + c][bL + j])
            //   A = T W:     A[bL + r][n] = sum_{j <= r} T[bL + r][bL + j] W[bL + j][n]
            // Items (row m or column n, block b) are independent and update only
            // their own L-segment.  Only the items the upper triangle needs are
            // computed: rows m < (b+1) L of block b in the first pass, columns
            // n >= b L in the second.  Each lane serves one block; a block gets
            // lanes in proportion to its items (SplitPlan), so every lane has at
            // most NIR (NIC) items.  The lane keeps its block of T in registers
            // (L <= 4) or reads it from LDS next to each item's loads.
            using SPl = SplitPlan<KP, LB, NT>;
            constexpr bool TREG = LB <= 4;
            Wt Tr_[TREG ? LB : 1][TREG ? LB : 1], Ti_[TREG ? LB : 1][TREG ? LB : 1];
            int b = 0, r0 = 0, nl = 1;
            bool sv = false;
            auto load_T = [&]() {
                if constexpr (TREG) {
#pragma unroll
                    for (int r = 0; r < LB; ++r)
#pragma unroll
                        for (int j = 0; j <= r; ++j) { Tr_[r][j] = sMr[(b * LB + r) * LB + j]; Ti_[r][j] = sMi[(b * LB + r) * LB + j]; }
                }
            };
            auto Tr = [&](int r, int j) -> Wt { if constexpr (TREG) return Tr_[r][j]; else return sMr[(b * LB + r) * LB + j]; };
            auto Ti = [&](int r, int j) -> Wt { if constexpr (TREG) return Ti_[r][j]; else return sMi[(b * LB + r) * LB + j]; };
            SPl::assign(tid, true, b, r0, nl, sv);
            load_T();
#pragma unroll
            for (int it = 0; it < SPl::NIR; ++it) {
                const int mi = r0 + it * nl;
                const bool need = sv && mi < (b + 1) * LB;
                const int m = need ? mi : 0;                // loads stay in the matrix
                Wt a_r[LB], a_i[LB];
#pragma unroll
                for (int j = 0; j < LB; ++j) { a_r[j] = sAr[m * LDA + b * LB + j]; a_i[j] = sAi[m * LDA + b * LB + j]; }
                Wt w_r[LB], w_i[LB];
#pragma unroll
                for (int c = 0; c < LB; ++c) {
                    Wt wr = 0, wi = 0;
#pragma unroll
                    for (int j = 0; j <= c; ++j) {          // w += a_j conj(T[c][j])
                        wr = fma(a_r[j], Tr(c, j), wr);
                        wr = fma(a_i[j], Ti(c, j), wr);
                        wi = fma(a_i[j], Tr(c, j), wi);
                        wi = fma(-a_r[j], Ti(c, j), wi);
                    }
                    w_r[c] = wr;
                    w_i[c] = wi;
                }
                if (need) {
#pragma unroll
                    for (int c = 0; c < LB; ++c) { sAr[m * LDA + b * LB + c] = w_r[c]; sAi[m * LDA + b * LB + c] = w_i[c]; }
                }
            }
            bsync();
            SPl::assign(tid, false, b, r0, nl, sv);
            load_T();
#pragma unroll
            for (int it = 0; it < SPl::NIC; ++it) {
                const int ni = b * LB + r0 + it * nl;
                const bool need = sv && ni < KP;
                const int nn = need ? ni : 0;
                Wt w_r[LB], w_i[LB];
#pragma unroll
                for (int j = 0; j < LB; ++j) { w_r[j] = sAr[(b * LB + j) * LDA + nn]; w_i[j] = sAi[(b * LB + j) * LDA + nn]; }
                Wt v_r[LB], v_i[LB];
#pragma unroll
                for (int r = 0; r < LB; ++r) {
                    Wt vr = 0, vi = 0;
#pragma unroll
                    for (int j = 0; j <= r; ++j) {          // v += T[r][j] w_j
                        vr = fma(Tr(r, j), w_r[j], vr);
                        vr = fma(-Ti(r, j), w_i[j], vr);
                        vi = fma(Tr(r, j), w_i[j], vi);
                        vi = fma(Ti(r, j), w_r[j], vi);
                    }
                    v_r[r] = vr;
                    v_i[r] = vi;
                }
                if (need) {
#pragma unroll
                    for (int r = 0; r < LB; ++r) { sAr[(b * LB + r) * LDA + nn] = v_r[r]; sAi[(b * LB + r) * LDA + nn] = v_i[r]; }
                }
            }
            bsync();
        }
    }

    if constexpr (LB == 0 && MODE == MODE_FULL && !C::AROW) {   // (AROW: from the Gram epilogue)
        if (P.gain && cblk == 0)
            for (int k = tid; k < K; k += NT) P.gain[ch * K + k] = (float)((Wt)1 - (Wt)s2 / sAr[k * LDA + k]);
    }

    // element (r, c) of the u_W matrix of the iteration: the Gram (stored whole),
    // or T A T^H (stored as its upper triangle; Hermitian with real diagonal)
    auto a_at = [&](int r, int c, Wt& re, Wt& im) {
        if constexpr (split) {
            const bool up = r <= c;
            const int o = up ? r * LDA + c : c * LDA + r;
            const Wt v = sAi[o];
            re = sAr[o];
            im = (r == c) ? (Wt)0 : (up ? v : -v);
        } else {
            re = sAr[r * LDA + c];
            im = sAi[r * LDA + c];
        }
    };

    // ------------------------------------------------------------ fp8 scale of the u_MV matrix
    // (a non-finite entry leaves the fp8 operand non-finite: FP8_SAT, as NONFINITE)
    if constexpr (FMT == F8 && !C::AROW) {            // (AROW: taken from the Gram accumulators)
        float ma = 0.f;
        bool nf = false;
        for (int i = tid; i < K * K; i += NT) {
            const int r = i / K, c = i % K;
            Wt re, im;
            a_at(r, c, re, im);
            ma = fmaxf(ma, fmaxf(fabsf((float)re), fabsf((float)im)));
            nf |= !__builtin_isfinite(re) || !__builtin_isfinite(im);
        }
        if (nf) myflag |= FLAG_FP8_SAT;
        ma = block_max(ma);
        eA = fp8_scale_exp(ma);
    }
    const float sA = ldexpf(1.f, eA);

    // ------------------------------------------------------------ u_MV operand of A
    // A-operand lane (g, n) of output tile phi holds row rowc(phi) (fixed per lane)
    // and the contraction values of source wave ws, block kb: columns colc(ws, kb, j).
    auto rowc = [&](int phi) -> int {
        int gm, im;
        O::cinv(n, gm, im);
        return (gm * NW + wave) * SH + 4 * phi + im;
    };
    // the same for the f64 shape used by the FP64 residual refresh
    auto rowc64 = [&](int phi) -> int {
        int gm, im;
        Op<F64, 1>::cinv(n, gm, im);
        return (gm * NW + wave) * SH + 4 * phi + im;
    };
    auto colc = [&](int ws, int kb, int j) -> int { return (g * NW + ws) * SH + kb * KPL + j; };
    auto fidx = [&](int phi, int ws, int kb, int ri) -> int { return ((phi * NW + ws) * NKB + kb) * 2 + ri; };
    frag afr[C::AREG ? C::NAV : 1];
    if constexpr (C::AREG || C::AFRAG_LDS) {
#pragma unroll
        for (int phi = 0; phi < NF; ++phi)
#pragma unroll
            for (int ws = 0; ws < NW; ++ws)
#pragma unroll
                for (int kb = 0; kb < NKB; ++kb) {
                    Wt vr[KPL], vi[KPL];
                    const int rr_ = rowc(phi);
#pragma unroll
                    for (int j = 0; j < KPL; ++j) a_at(rr_, colc(ws, kb, j), vr[j], vi[j]);
                    const frag fr = O::pack(vr, sA), fi = O::pack(vi, sA);
                    if constexpr (C::AREG) {
                        afr[fidx(phi, ws, kb, 0)] = fr;
                        afr[fidx(phi, ws, kb, 1)] = fi;
                    } else {
                        sF[fidx(phi, ws, kb, 0) * NT + tid] = fr;
                        sF[fidx(phi, ws, kb, 1) * NT + tid] = fi;
                    }
                }
    }
    if constexpr (NW > 1) {
        if (x_in_gram) __syncthreads();               // every wave has packed before x overwrites the Gram
    }
    if (compact) {
        // B into the Gram's slot, next to x (the packing above has read A)
        bsync();
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (NW == 1 || f % NW == wave) {
                const int s = f / NW;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int row = 16 * f + OG::crow(g, jj);
                    sBr[row * 16 + n] = bcr[s][jj];
                    sBi[row * 16 + n] = bci[s][jj];
                }
            }
        }
        bsync();
    }
    auto A_op = [&](int phi, int ws, int kb, int ri) -> frag {
        if constexpr (C::AREG) {
            return afr[fidx(phi, ws, kb, ri)];
        } else if constexpr (C::AFRAG_LDS) {
            return sF[fidx(phi, ws, kb, ri) * NT + tid];
        } else if constexpr (C::AROW) {
            // KPL consecutive contraction values of one row: one aligned LDS read
            const unsigned char* base = ri ? sA8i : sA8r;
            return *reinterpret_cast<const frag*>(base + ((size_t)rowc(phi) * KP + colc(ws, kb, 0)) * C::ESZ);
        } else {
            Wt re, im;
            a_at(rowc(phi), colc(ws, kb, 0), re, im);
            const Wt v = ri ? im : re;
            return O::pack(&v, 1.f);
        }
    };

    // ------------------------------------------------------------ helpers for the solve
    int parity = 0;
    // sum of per-lane partials over the column (lane groups, then waves in order);
    // up to four values at once
    auto col_reduce = [&](Wt* v, int cnt) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < cnt) v[k] = col_sum(v[k]);
        if constexpr (NW > 1) {
            Wt* red = sRed + parity * NW * 16 * 4;
            if (g == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < cnt) red[(wave * 16 + n) * 4 + k] = v[k];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < cnt) {
                    Wt s = red[(0 * 16 + n) * 4 + k];
#pragma unroll
                    for (int w = 1; w < NW; ++w) s = s + red[(w * 16 + n) * 4 + k];
                    v[k] = s;
                }
            }
            parity ^= 1;
        }
    };
    // publish this wave's slots of p (NW > 1) so that other waves can read them
    auto publish = [&](const Wt* vr, const Wt* vi) {
        if constexpr (NW > 1) {
            Wt* dst = sXP + ((size_t)wave * 64 + lane) * 2 * SH;
#pragma unroll
            for (int e = 0; e < SH; ++e) { dst[e] = vr[e]; dst[SH + e] = vi[e]; }
        }
    };
    auto fetch = [&](int ws, int e, int part) -> Wt {
        return sXP[((size_t)ws * 64 + lane) * 2 * SH + part * SH + e];
    };

    const int base_c = (g * NW + wave) * SH;
    // z = M r (block-diagonal, lane-local, u_W)
    auto apply_M = [&](const Wt* rr, const Wt* ri, Wt* zr, Wt* zi) {
        if constexpr (LB > 0) {
#pragma unroll
            for (int e = 0; e < SH; ++e) {
                const int j0 = (e / LB) * LB;
                const int c = base_c + e;
                Wt ar = 0, ai = 0;
#pragma unroll
                for (int j = 0; j < LB; ++j) {
                    const Wt mr = sMr[c * LB + j], mi = sMi[c * LB + j];
                    ar = fma(mr, rr[j0 + j], ar);
                    ar = fma(-mi, ri[j0 + j], ar);
                    ai = fma(mr, ri[j0 + j], ai);
                    ai = fma(mi, rr[j0 + j], ai);
                }
                zr[e] = ar;
                zi[e] = ai;
            }
        } else {
#pragma unroll
            for (int e = 0; e < SH; ++e) { zr[e] = rr[e]; zi[e] = ri[e]; }
        }
    };
    // v <- T v (b_bar = T b) and v <- T^H v (x = T^H x_bar), lane-local, in arithmetic type Ta
    auto apply_T = [&](auto* vr, auto* vi) {
        using Ta = typename std::remove_reference<decltype(vr[0])>::type;
        if constexpr (LB > 0) {
#pragma unroll
            for (int b0 = 0; b0 < SH; b0 += LB) {
                Ta ur[LB], ui[LB];
#pragma unroll
                for (int r = 0; r < LB; ++r) {
                    const int c = base_c + b0 + r;
                    Ta sr = 0, si = 0;
#pragma unroll
                    for (int j = 0; j <= r; ++j) {
                        const Ta t_r = (Ta)sMr[c * LB + j], t_i = (Ta)sMi[c * LB + j];
                        sr = fma(t_r, vr[b0 + j], sr);
                        sr = fma(-t_i, vi[b0 + j], sr);
                        si = fma(t_r, vi[b0 + j], si);
                        si = fma(t_i, vr[b0 + j], si);
                    }
                    ur[r] = sr;
                    ui[r] = si;
                }
#pragma unroll
                for (int r = 0; r < LB; ++r) { vr[b0 + r] = ur[r]; vi[b0 + r] = ui[r]; }
            }
        }
    };
    auto apply_TH = [&](auto* vr, auto* vi) {
        using Ta = typename std::remove_reference<decltype(vr[0])>::type;
        if constexpr (LB > 0) {
#pragma unroll
            for (int b0 = 0; b0 < SH; b0 += LB) {
                Ta ur[LB], ui[LB];
                const int cb0 = base_c + b0;
#pragma unroll
                for (int r = 0; r < LB; ++r) {
                    Ta sr = 0, si = 0;
#pragma unroll
                    for (int j = r; j < LB; ++j) {          // += conj(T[j][r]) v_j
                        const Ta t_r = (Ta)sMr[(cb0 + j) * LB + r], t_i = (Ta)sMi[(cb0 + j) * LB + r];
                        sr = fma(t_r, vr[b0 + j], sr);
                        sr = fma(t_i, vi[b0 + j], sr);
                        si = fma(t_r, vi[b0 + j], si);
                        si = fma(-t_i, vr[b0 + j], si);
                    }
                    ur[r] = sr;
                    ui[r] = si;
                }
#pragma unroll
                for (int r = 0; r < LB; ++r) { vr[b0 + r] = ur[r]; vi[b0 + r] = ui[r]; }
            }
        }
    };

    // flags raised so far, made wave-uniform (scalar registers) so that no
    // vector register holds them through the solve
    uint32_t wflag = 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        if (__ballot((myflag >> b) & 1u) != 0) wflag |= 1u << b;
    myflag = 0u;
    const int passes = REF ? 1 + P.refine_steps : 1;   // REF: built with FP64 refinement
    int es = 0;                                       // exponent of the current pass's residual scale
    for (int pass = 0; pass < passes; ++pass) {
        if (pass > 0) {
            // -------------------------------------------- FP64 residual through H
            double resr[SH], resi[SH], x64r[SH], x64i[SH];
#pragma unroll
            for (int e = 0; e < SH; ++e) {
                resr[e] = 0; resi[e] = 0;
                x64r[e] = sX64r[e * NT + tid];
                x64i[e] = sX64i[e * NT + tid];
            }
            if constexpr (NW == 1) {
                // one antenna at a time: e_a = y_a - h_a x (column sums), res += conj(h_a) e_a
#pragma unroll 1
                for (int a = 0; a < Nbs; ++a) {
                    double hr[SH], hi[SH];
                    double sr = 0, si = 0;
#pragma unroll
                    for (int e = 0; e < SH; ++e) {
                        const int c = base_c + e;
                        CxB<IOT>::load(bH, hofs(a, c), hr[e], hi[e]);
                        sr = fma(hr[e], x64r[e], sr);
                        sr = fma(-hi[e], x64i[e], sr);
                        si = fma(hr[e], x64i[e], si);
                        si = fma(hi[e], x64r[e], si);
                    }
                    sr = col_sum(sr);
                    si = col_sum(si);
                    double yr, yi;
                    CxB<IOT>::load(bY, yofs(a), yr, yi);
                    const double vr = yr - sr, vi = yi - si;
#pragma unroll
                    for (int e = 0; e < SH; ++e) {
                        resr[e] = fma(hr[e], vr, resr[e]);
                        resr[e] = fma(hi[e], vi, resr[e]);
                        resi[e] = fma(hr[e], vi, resi[e]);
                        resi[e] = fma(-hi[e], vr, resi[e]);
                    }
                }
            } else {
                // chunks of RC antennas: per-wave column partials through LDS
#pragma unroll 1
                for (int a0 = 0; a0 < Nbs; a0 += C::RC) {
#pragma unroll 1
                    for (int u = 0; u < C::RC; ++u) {
                        const int a = a0 + u;
                        double sr = 0, si = 0;
#pragma unroll
                        for (int e = 0; e < SH; ++e) {
                            const int c = base_c + e;
                            double hr, hi;
                            CxB<IOT>::load(bH, hofs(a, c), hr, hi);
                            sr = fma(hr, x64r[e], sr);
                            sr = fma(-hi, x64i[e], sr);
                            si = fma(hr, x64i[e], si);
                            si = fma(hi, x64r[e], si);
                        }
                        sr = col_sum(sr);
                        si = col_sum(si);
                        if (g == 0) {
                            sRef[((wave * C::RC + u) * 16 + n) * 2 + 0] = sr;
                            sRef[((wave * C::RC + u) * 16 + n) * 2 + 1] = si;
                        }
                    }
                    __syncthreads();
#pragma unroll 1
                    for (int u = 0; u < C::RC; ++u) {
                        const int a = a0 + u;
                        if (a >= Nbs) break;
                        double er = sRef[((0 * C::RC + u) * 16 + n) * 2 + 0];
                        double ei = sRef[((0 * C::RC + u) * 16 + n) * 2 + 1];
#pragma unroll
                        for (int w = 1; w < NW; ++w) {
                            er += sRef[((w * C::RC + u) * 16 + n) * 2 + 0];
                            ei += sRef[((w * C::RC + u) * 16 + n) * 2 + 1];
                        }
                        double yr, yi;
                        CxB<IOT>::load(bY, yofs(a), yr, yi);
                        const double vr = yr - er, vi = yi - ei;
#pragma unroll
                        for (int e = 0; e < SH; ++e) {
                            const int c = base_c + e;
                            double hr, hi;
                            CxB<IOT>::load(bH, hofs(a, c), hr, hi);
                            resr[e] = fma(hr, vr, resr[e]);
                            resr[e] = fma(hi, vi, resr[e]);
                            resi[e] = fma(hr, vi, resi[e]);
                            resi[e] = fma(-hi, vr, resi[e]);
                        }
                    }
                    __syncthreads();
                }
            }
            double cm = 0;
#pragma unroll
            for (int e = 0; e < SH; ++e) {
                resr[e] = fma(-s2, x64r[e], resr[e]);
                resi[e] = fma(-s2, x64i[e], resi[e]);
                if (base_c + e >= K || !colv) { resr[e] = 0; resi[e] = 0; }
                cm = fmax(cm, fmax(fabs(resr[e]), fabs(resi[e])));
            }
            // per-column power-of-two scale: max |r| lands in [1, 2)
            cm = col_max(cm);
            if constexpr (NW > 1) {
                __syncthreads();
                if (g == 0) sRef[wave * 16 + n] = cm;
                __syncthreads();
                double mm = sRef[n];
#pragma unroll
                for (int w = 1; w < NW; ++w) mm = fmax(mm, sRef[w * 16 + n]);
                cm = mm;
                __syncthreads();
            }
            es = 0;
            if (cm > 0 && __builtin_isfinite(cm)) {
                int ex;
                frexp(cm, &ex);
                es = ex - 1;
                es = es < -126 ? -126 : (es > 126 ? 126 : es);
            }
            const double sc = ldexp(1.0, -es);
#pragma unroll
            for (int e = 0; e < SH; ++e) { resr[e] *= sc; resi[e] *= sc; }
            if constexpr (split) apply_T(resr, resi);   // b_bar = T (r sc), FP64 arithmetic
#pragma unroll
            for (int e = 0; e < SH; ++e) {
                const int c = base_c + e;
                sBr[c * 16 + n] = (Wt)resr[e];
                sBi[c * 16 + n] = (Wt)resi[e];
            }
            bsync();
        }

        // ------------------------------------------------ 3. (P)CG
        // x of this pass: in registers where it fits beside the other vectors
        // (stored to LDS only for an FP64 refresh), else accumulated in LDS
        // (FP64: measured no faster in registers, and it spills more)
        constexpr bool xreg = SH * sizeof(Wt) <= 32 && FMT != F64;
        Wt rr[SH], ri[SH], pr[SH], pi[SH], xr_[SH], xi_[SH];
        {
            Wt wr[SH], wi[SH];
#pragma unroll
            for (int e = 0; e < SH; ++e) {
                xr_[e] = 0;
                xi_[e] = 0;
                if constexpr (!xreg) {
                    sXr[e * NT + tid] = 0;
                    sXi[e * NT + tid] = 0;
                }
                rr[e] = sBr[(base_c + e) * 16 + n];
                ri[e] = sBi[(base_c + e) * 16 + n];
            }
            if (split && pass == 0) {
                apply_T(rr, ri);                        // b_bar = T b, kept for the FP64 refresh
#pragma unroll
                for (int e = 0; e < SH; ++e) { sBr[(base_c + e) * 16 + n] = rr[e]; sBi[(base_c + e) * 16 + n] = ri[e]; }
            }
            if constexpr (left) apply_M(rr, ri, wr, wi);   // p0 = M r0 (Alg. 3) or r0
            else {
#pragma unroll
                for (int e = 0; e < SH; ++e) { wr[e] = rr[e]; wi[e] = ri[e]; }
            }
#pragma unroll
            for (int e = 0; e < SH; ++e) { pr[e] = wr[e]; pi[e] = wi[e]; }
        }
        Wt rho_cur;
        {
            Wt v[4];
            v[0] = 0;
#pragma unroll
            for (int e = 0; e < SH; ++e) { v[0] = fma(rr[e], pr[e], v[0]); v[0] = fma(ri[e], pi[e], v[0]); }
            col_reduce(v, 1);
            rho_cur = v[0];                            // r0^H r0 (Alg. 2) / r0^H z0 (textbook PCG)
        }
        bool live = true, broken = false;
        int eP = 0;
        for (int it = 1; it <= P.iters; ++it) {
            // ---- varpi = A p   [u_MV]
            if constexpr (NW > 1) {
                __syncthreads();
                publish(pr, pi);
                __syncthreads();
            }
            if constexpr (FMT == F8) {
                float am = 0.f;
#pragma unroll
                for (int e = 0; e < SH; ++e) am = fmaxf(am, fmaxf(fabsf(pr[e]), fabsf(pi[e])));
                eP = fp8_scale_exp(column_max(am));
            }
            const float sP = ldexpf(1.f, eP);
            acc_t Wr_[NF], Wi_[NF];
#pragma unroll
            for (int phi = 0; phi < NF; ++phi) { Wr_[phi] = acc_t{0, 0, 0, 0}; Wi_[phi] = acc_t{0, 0, 0, 0}; }
            if constexpr (FMT == F64) {
                // FP64: three real products per complex one, Re = P1 - P2 and
                // Im = P3 - P1 - P2 for P1 = a_r p_r, P2 = a_i p_i,
                // P3 = (a_r + a_i)(p_r + p_i); P1 and P2 accumulate in Wr_ and Wi_
                acc_t P3[NF];
#pragma unroll
                for (int phi = 0; phi < NF; ++phi) P3[phi] = acc_t{0, 0, 0, 0};
#pragma unroll
                for (int ws = 0; ws < NW; ++ws) {
#pragma unroll
                    for (int kb = 0; kb < NKB; ++kb) {
                        Wt vr[KPL], vi[KPL];
#pragma unroll
                        for (int j = 0; j < KPL; ++j) {
                            const int e = kb * KPL + j;
                            if (NW == 1 || ws == wave) { vr[j] = pr[e]; vi[j] = pi[e]; }
                            else { vr[j] = fetch(ws, e, 0); vi[j] = fetch(ws, e, 1); }
                        }
                        const frag Br = O::pack(vr, sP), Bi = O::pack(vi, sP);
#pragma unroll
                        for (int phi = 0; phi < NF; ++phi) {
                            const frag a_r = A_op(phi, ws, kb, 0), a_i = A_op(phi, ws, kb, 1);
                            frag a_s = a_r;
                            asm("" : "+v"(a_s) : "s"(it));  // the sum is formed here, not hoisted into registers
                            Wr_[phi] = O::mfma(a_r, Br, Wr_[phi]);
                            Wi_[phi] = O::mfma(a_i, Bi, Wi_[phi]);
                            P3[phi] = O::mfma(a_s + a_i, Br + Bi, P3[phi]);
                        }
                    }
                }
#pragma unroll
                for (int phi = 0; phi < NF; ++phi)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const double p1 = Wr_[phi][jj], p2 = Wi_[phi][jj];
                        Wr_[phi][jj] = p1 - p2;
                        Wi_[phi][jj] = (P3[phi][jj] - p1) - p2;
                    }
            } else {
#pragma unroll
                for (int ws = 0; ws < NW; ++ws) {
#pragma unroll
                    for (int kb = 0; kb < NKB; ++kb) {
                        Wt vr[KPL], vi[KPL];
#pragma unroll
                        for (int j = 0; j < KPL; ++j) {
                            const int e = kb * KPL + j;
                            if (NW == 1 || ws == wave) { vr[j] = pr[e]; vi[j] = pi[e]; }
                            else { vr[j] = fetch(ws, e, 0); vi[j] = fetch(ws, e, 1); }
                        }
                        const frag Br = O::pack(vr, sP), Bi = O::pack(vi, sP), nBi = O::neg(Bi);
#pragma unroll
                        for (int phi = 0; phi < NF; ++phi) {
                            const frag a_r = A_op(phi, ws, kb, 0), a_i = A_op(phi, ws, kb, 1);
                            Wr_[phi] = O::mfma(a_r, Br, Wr_[phi]);
                            Wr_[phi] = O::mfma(a_i, nBi, Wr_[phi]);
                            Wi_[phi] = O::mfma(a_i, Br, Wi_[phi]);
                            Wi_[phi] = O::mfma(a_r, Bi, Wi_[phi]);
                        }
                    }
                }
            }
            Wt wr[SH], wi[SH];
            const Wt inv_s = (Wt)(ldexpf(1.f, -eA)), inv_p = (Wt)(ldexpf(1.f, -eP));
#pragma unroll
            for (int phi = 0; phi < NF; ++phi)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    Wt a = (Wt)Wr_[phi][jj], b = (Wt)Wi_[phi][jj];
                    if constexpr (FMT == F8) { a = a * inv_s * inv_p; b = b * inv_s * inv_p; }
                    wr[4 * phi + jj] = a;
                    wi[4 * phi + jj] = b;
                }
            // ---- phi = p^H varpi, rho_{i-1}  [u_IP]
            Wt v[4];
            v[0] = 0; v[1] = 0;
            const bool need_rp = left && (P.variant == 0);
#pragma unroll
            for (int e = 0; e < SH; ++e) {
                v[0] = fma(pr[e], wr[e], v[0]);
                v[0] = fma(pi[e], wi[e], v[0]);
            }
            if (need_rp) {
#pragma unroll
                for (int e = 0; e < SH; ++e) {
                    v[1] = fma(rr[e], pr[e], v[1]);
                    v[1] = fma(ri[e], pi[e], v[1]);
                }
            }
            col_reduce(v, need_rp ? 2 : 1);
            const Wt ph = v[0];
            const Wt rho_prev = need_rp ? v[1] : rho_cur;
            // ---- guard, alpha, x and r updates  [u_W]
            const bool ok = live && __builtin_isfinite(ph) && __builtin_isfinite(rho_prev) && ph > 0 && rho_prev > 0;
            if (live && !ok && colv) broken = true;
            live = ok;
            Wt alpha_rec = 0, beta_rec = 0;             // the step's coefficients (0 once frozen)
            if (live) {
                const Wt alpha = rho_prev / ph;
                alpha_rec = alpha;
                if constexpr (!xreg) {
#pragma unroll
                    for (int e = 0; e < SH; ++e) { xr_[e] = sXr[e * NT + tid]; xi_[e] = sXi[e * NT + tid]; }
                }
#pragma unroll
                for (int e = 0; e < SH; ++e) {
                    xr_[e] = fma(alpha, pr[e], xr_[e]);
                    xi_[e] = fma(alpha, pi[e], xi_[e]);
                    rr[e] = fma(-alpha, wr[e], rr[e]);
                    ri[e] = fma(-alpha, wi[e], ri[e]);
                }
                if constexpr (!xreg) {
#pragma unroll
                    for (int e = 0; e < SH; ++e) { sXr[e * NT + tid] = xr_[e]; sXi[e * NT + tid] = xi_[e]; }
                }
            }
            // ---- FP64 residual refresh on the stored Gram (A, or T A T^H)
            // (not built for AROW: no u_W Gram is kept; refused on the host)
            if (!C::AROW && P.refresh_every > 0 && it % P.refresh_every == 0 && it < P.iters) {
                if constexpr (xreg) {
#pragma unroll
                    for (int e = 0; e < SH; ++e) { sXr[e * NT + tid] = xr_[e]; sXi[e * NT + tid] = xi_[e]; }
                }
                if constexpr (NW > 1) __syncthreads();   // x of every wave visible
                // three real products per complex one: Re = P1 - P2 and
                // Im = P3 - P1 - P2 for P1 = a_r x_r, P2 = a_i x_i,
                // P3 = (a_r + a_i)(x_r + x_i)
                f64x4 Rr[NF], Ri[NF], R3[NF];
#pragma unroll
                for (int phi = 0; phi < NF; ++phi) {
                    Rr[phi] = f64x4{0, 0, 0, 0}; Ri[phi] = f64x4{0, 0, 0, 0}; R3[phi] = f64x4{0, 0, 0, 0};
                }
#pragma unroll
                for (int ws = 0; ws < NW; ++ws) {
#pragma unroll
                    for (int kb = 0; kb < SH; ++kb) {
                        const double bx = (double)sXr[kb * NT + ws * 64 + lane];
                        const double by = (double)sXi[kb * NT + ws * 64 + lane];
                        const int cc = (g * NW + ws) * SH + kb;
#pragma unroll
                        for (int phi = 0; phi < NF; ++phi) {
                            Wt are, aim;
                            a_at(rowc64(phi), cc, are, aim);
                            const double a_r = (double)are, a_i = (double)aim;
                            Rr[phi] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r, bx, Rr[phi], 0, 0, 0);
                            Ri[phi] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i, by, Ri[phi], 0, 0, 0);
                            R3[phi] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r + a_i, bx + by, R3[phi], 0, 0, 0);
                        }
                    }
                }
                if (live) {
#pragma unroll
                    for (int phi = 0; phi < NF; ++phi)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const int e = 4 * phi + jj;
                            const double b_r = (double)sBr[(base_c + e) * 16 + n];
                            const double b_i = (double)sBi[(base_c + e) * 16 + n];
                            const double p1 = Rr[phi][jj], p2 = Ri[phi][jj];
                            rr[e] = (Wt)(b_r - (p1 - p2));
                            ri[e] = (Wt)(b_i - ((R3[phi][jj] - p1) - p2));
                        }
                }
                if constexpr (NW > 1) __syncthreads();   // before x changes again
                if constexpr (xreg) {
                    // reloaded, so that x is not held in registers across the refresh
#pragma unroll
                    for (int e = 0; e < SH; ++e) { xr_[e] = sXr[e * NT + tid]; xi_[e] = sXi[e * NT + tid]; }
                }
            }
            // ---- z = M r (left form) or r, rho_i, beta, p
            Wt zr[SH], zi[SH];
            if constexpr (left) apply_M(rr, ri, zr, zi);
            else {
#pragma unroll
                for (int e = 0; e < SH; ++e) { zr[e] = rr[e]; zi[e] = ri[e]; }
            }
            v[0] = 0;
#pragma unroll
            for (int e = 0; e < SH; ++e) { v[0] = fma(rr[e], zr[e], v[0]); v[0] = fma(ri[e], zi[e], v[0]); }
            col_reduce(v, 1);
            const Wt rho_new = v[0];
            if (live) {
                const Wt beta = rho_new / rho_prev;
                beta_rec = beta;
#pragma unroll
                for (int e = 0; e < SH; ++e) {
                    pr[e] = fma(beta, pr[e], zr[e]);
                    pi[e] = fma(beta, pi[e], zi[e]);
                }
            }
            rho_cur = rho_new;
            if (MODE == MODE_FULL && P.ab_hist && pass == 0 && g == 0 && wave == 0 && colv && col < KAPPA_COLS) {
                // one lane per recorded received-vector column writes alpha_i, beta_i
                const int nrec = R < KAPPA_COLS ? R : KAPPA_COLS;
                float* h = P.ab_hist + (((int64_t)blockIdx.x * nrec + col) * P.iters + (it - 1)) * 2;
                h[0] = (float)alpha_rec;
                h[1] = (float)beta_rec;
            }
        }
        if (broken) myflag |= FLAG_BREAKDOWN;
        // ------------------------------------------------ back-transform and refinement bookkeeping
        if (pass == 0) {
            Wt xo_r[SH], xo_i[SH];
#pragma unroll
            for (int e = 0; e < SH; ++e) {
                xo_r[e] = xreg ? xr_[e] : sXr[e * NT + tid];
                xo_i[e] = xreg ? xi_[e] : sXi[e * NT + tid];
            }
            if constexpr (split) apply_TH(xo_r, xo_i);  // x = T^H x_bar  (u_W)
            if (REF && P.refine_steps > 0) {
#pragma unroll
                for (int e = 0; e < SH; ++e) { sX64r[e * NT + tid] = (double)xo_r[e]; sX64i[e * NT + tid] = (double)xo_i[e]; }
            } else {
                // ---- 5. slicer + stores (no refinement); padded rows and
                // columns fall outside the output ranges and are dropped
                const Wt nu = (Wt)P.nu, mm = (Wt)P.m;
                out_begin();
#pragma unroll
                for (int e = 0; e < SH; ++e)
                    store_out(base_c + e, xo_r[e], xo_i[e], slice_label<Wt>(xo_r[e], xo_i[e], nu, mm, P.m, P.bits));
                out_end();
            }
        } else {
            double dr[SH], di[SH];
#pragma unroll
            for (int e = 0; e < SH; ++e) {
                dr[e] = (double)(xreg ? xr_[e] : sXr[e * NT + tid]);
                di[e] = (double)(xreg ? xi_[e] : sXi[e * NT + tid]);
            }
            if constexpr (split) apply_TH(dr, di);      // d = T^H d_bar  (FP64 arithmetic)
            const double us = ldexp(1.0, es);          // x += d / sc, exact scaling
#pragma unroll
            for (int e = 0; e < SH; ++e) {
                sX64r[e * NT + tid] = sX64r[e * NT + tid] + dr[e] * us;
                sX64i[e * NT + tid] = sX64i[e * NT + tid] + di[e] * us;
            }
        }
        if constexpr (NW > 1) __syncthreads();
    }

    // ------------------------------------------------------------ 5. slicer + stores (refined, FP64)
    if (REF && P.refine_steps > 0) {
        const double nu = P.nu, mm = (double)P.m;
        out_begin();
#pragma unroll
        for (int e = 0; e < SH; ++e) {
            const double xr = sX64r[e * NT + tid], xi = sX64i[e * NT + tid];
            store_out(base_c + e, xr, xi, slice_label<double>(xr, xi, nu, mm, P.m, P.bits));
        }
        out_end();
    }
    myflag |= wflag;
    const bool one_block = P.R <= 16;                  // the only workgroup / item of this channel
    if constexpr (MODE == MODE_FULL) {
        if (myflag) atomicOr(&sFlag, myflag);
        __syncthreads();
        if (tid == 0 && P.flags) {
            if (one_block) P.flags[ch] = sFlag;
            else if (sFlag) atomicOr(&P.flags[ch], sFlag);     // flags were cleared before the launch
        }
    } else {
        uint32_t f = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (__ballot((myflag >> b) & 1u) != 0) f |= 1u << b;
        if (tid == 0 && P.flags) {
            if (one_block) P.flags[ch] = f;
            else if (f) atomicOr(&P.flags[ch], f);
        }
    }
}

// Register budget of a one-workgroup-per-channel build, in waves per SIMD:
// four where the allocation fits 128 registers without spilling (measured:
// K <= 32, fp16 / bf16 operands, symmetric L = 4, complex64 I/O), three for
// the other K <= 32 reduced-precision and FP32 builds, two for FP64 at
// K <= 32 (a few registers spill, and it still measured 13 % faster than one
// wave), no constraint for FP64 at K = 64, K = 128 and refinement builds.
// Four-wave channels (K = 64) ask for two waves per SIMD: two channels per CU.
template <int KP, int NW, int FMT, int LB, bool SPLIT, bool REF, typename IOT> constexpr int fused_waves() {
    if (REF) return 1;
    if (NW >= 4) return 2;
    if (FMT == F64 && KP == 32) return 2;
    if (KP == 32 && (FMT == F16 || FMT == BF16) && LB == 4 && SPLIT && sizeof(IOT) == 4) return 4;
    return Cfg<KP, 1, FMT, LB>::MIN_WAVES;
}

template <int KP, int NW, int FMT, int LB, bool SPLIT, bool REF, typename IOT>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(fused_waves<KP, NW, FMT, LB, SPLIT, REF, IOT>())))
void fused_kernel(const FusedParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    int64_t ch = blockIdx.x;
    if (P.chan_idx) {
        ch = P.chan_idx[blockIdx.x];                  // uniform: the whole workgroup skips together
        if (ch < 0 || ch >= P.B) return;
    }
    detect_channel<KP, NW, FMT, LB, SPLIT, REF, IOT, MODE_FULL>(P, ch, blockIdx.y, smem, smem, nullptr, threadIdx.x);
}

// Pipelined form for one-wave channels: a persistent workgroup of two waves
// walks its items (channel, block of received vectors) in steps; in step k
// wave 0 forms the Gram and matched filter of item k+1 into one LDS buffer
// while wave 1 solves item k from the other, so the HBM stream of the Gram
// overlaps the on-chip solve.  LDS: [buffer 0 | buffer 1 | solver regions].
template <int KP, int FMT, int LB> struct PipeCfg {
    using C = Cfg<KP, 1, FMT, LB>;
    static constexpr size_t BUF = C::off_M;           // [Ar | Ai | Br | Bi]
    __host__ __device__ static constexpr size_t lds(bool split, int refresh_every) {
        return BUF + C::lds_general(split, false, refresh_every);
    }
};

template <int KP, int FMT, int LB, bool SPLIT, typename IOT>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(Cfg<KP, 1, FMT, LB>::MIN_WAVES)))
void pipe_kernel(const FusedParams P) {
    constexpr size_t BUF = PipeCfg<KP, FMT, LB>::BUF;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t gflag[2];
    // the role is uniform per wave: a scalar branch, so the roles' code never shares registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane0 = threadIdx.x & 63;
    const int ncb = (P.R + 15) / 16;
    const int64_t items = P.B * ncb, G = gridDim.x;
    int64_t it = blockIdx.x;
    // the buffer of each role is a compile-time offset in both halves of a
    // step pair, so LDS addresses fold into the instructions' offsets
    auto step = [&](auto cur_c) {
        constexpr int cur = decltype(cur_c)::value, nxt = cur ^ 1;
        // an opaque copy of the lane index per step keeps the compiler from
        // hoisting every lane-dependent address of both roles out of the loop
        // (they would stay live across the whole loop and spill)
        int lane = lane0;
        asm volatile("" : "+v"(lane));
        if (wave == 0) {
            const int64_t nit = it + G;
            if (nit < items)
                detect_channel<KP, 1, FMT, LB, SPLIT, false, IOT, MODE_GRAM>(P, nit / ncb, (int)(nit % ncb),
                                                                              smem + nxt * BUF, smem + BUF,
                                                                              &gflag[nxt], lane);
        } else {
            detect_channel<KP, 1, FMT, LB, SPLIT, false, IOT, MODE_SOLVE>(P, it / ncb, (int)(it % ncb),
                                                                           smem + cur * BUF, smem + BUF,
                                                                           &gflag[cur], lane);
        }
        __syncthreads();
        it += G;
    };
    if (wave == 0 && it < items)
        detect_channel<KP, 1, FMT, LB, SPLIT, false, IOT, MODE_GRAM>(P, it / ncb, (int)(it % ncb), smem, smem + BUF,
                                                                      &gflag[0], lane0);
    __syncthreads();
    // the loop bound depends on blockIdx only, so both waves meet every barrier
    while (it < items) {
        step(std::integral_constant<int, 0>{});
        if (it >= items) break;
        step(std::integral_constant<int, 1>{});
    }
}

}  // namespace fpcg
