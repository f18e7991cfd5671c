// The register-resident ("slab") detector kernel for K = 64 and K = 128.
//
// One workgroup of NW = K/16 waves handles one channel and one block of up to
// 16 received vectors.  Wave w owns slab w: rows 16w .. 16w+15 of every
// iterate (x, r, p, b) and columns 16w .. 16w+15 of the iteration matrix A.
// Lane (g, n) of a wave holds, in the output layout of the fp32-accumulating
// 16x16 matrix-core tiles, rows 4g + i (i < 4) of its slab and received-vector
// column n; for A, rows 16f + 4g + i of column 16w + n for every row slab f.
//
//   1. Gram and matched filter (Sec. II, eq. inversion) on the matrix cores:
//      the upper-triangle 16x16 tiles of A = H^H H + sigma^2 I are spread over
//      the waves; every tile goes through LDS once and each wave reads its
//      column slab back (tiles below the diagonal as conjugate transposes).
//   2. Block-Jacobi setup (eq. pre_BJ).  L = 4: Cholesky of every 4 x 4
//      diagonal block, T = C^{-1}; the symmetric form (the system of Thm 4)
//      rewrites A <- T A T^H and b <- T b in registers (rows lane-local, columns
//      across four adjacent lanes); Alg. 3 as printed keeps M_d = T^H T.
//      L = 8 and 16 (symmetric form): the blocks tile the diagonal 16 x 16
//      tiles; each wave factors those of its own tile, and every upper tile
//      is rewritten in LDS as T_a A_ab T_b^H on the fp32 matrix cores before
//      the waves read their column slabs.
//   3. (P)CG (Alg. 2 / Alg. 3): A p on the matrix cores with A's operand copy
//      in registers -- A p for rows of slab w contracts A's row slab w, which is
//      the conjugate of the column slab the wave holds, so every operand
//      fragment is the lane's own value -- and p of every slab read from LDS
//      (each wave publishes its own slab once per iteration).  Inner products
//      are lane-local sums reduced over the lane groups and then over the
//      waves in a fixed order.  The FP64 refresh r = b - A x uses the FP64
//      matrix cores on the u_W copy of A, also in registers.
//   4. Slicer epilogue; outputs staged in LDS and stored as whole chunks.
//
// The FP64 matrix core's output tile puts row 4i + g (not 4g + i) in lane
// group g, element i; the FP64 operand copies of A hold column rho(n) in lane
// n (rho(4i + g) = 4g + i) instead of column n, so its products land in the
// same layout as the others.
#pragma once

#include "fpcg_fused.hpp"

namespace fpcg {

// row of a 16-row tile that the FP64 matrix core's output position m holds
// when the operand's lane n carries row rho(n): rho(4i + g) = 4g + i
__device__ __forceinline__ int rho16(int m) { return 4 * (m & 3) + (m >> 2); }

template <int KP_, int FMT_, int LB_> struct SlabCfg {
    static constexpr int KP = KP_, FMT = FMT_, LB = LB_;
    static_assert(KP == 64 || KP == 128, "slab kernel: K = 64 or 128");
    static_assert(FMT == F64 || FMT == F32 || FMT == F16 || FMT == BF16, "slab kernel: no fp8");
    static_assert(LB == 0 || LB == 4 || LB == 8 || LB == 16, "slab kernel: L = 0, 4, 8 or 16");
    static constexpr int NW = KP / 16, F = KP / 16, NT = 64 * NW;
    static constexpr bool LOWP = (FMT == F16 || FMT == BF16);
    using Wt = typename std::conditional<FMT == F64, double, float>::type;
    static constexpr size_t W = sizeof(Wt);
    // A p: fp16/bf16 16x16x32 over two row slabs; fp32 / fp64 16x16x4 over (slab, element)
    static constexpr int KPL = LOWP ? 8 : 1;
    using O = Op<FMT, KPL>;
    using frag = typename O::frag;
    // Gram / matched filter operands per lane and instruction, instructions per loaded block
    static constexpr int KPLG = LOWP ? 8 : 1;
    static constexpr int NSUB = LOWP ? 1 : (F <= 4 ? 4 : 2);
    static constexpr int NLD = KPLG * NSUB;
    static constexpr int KBG = 4 * NLD;               // antennas per loaded block
    using OG = Op<FMT, KPLG>;
    static constexpr int NTILE = F * (F + 1) / 2;
    static constexpr int PPW = (NTILE + NW - 1) / NW;
    // LDS: [main: Gram tiles, then the p / x exchange, then the staged outputs]
    //      [D: diagonal blocks] [T: T blocks, then M_d for the left form] [red]
    // a tile plane in LDS: 16 rows of TR words (padded, so that reads down a
    // column -- transposed tiles, the tile transform's operands -- are free of
    // bank conflicts)
    static constexpr int TR = 17, TP = 16 * TR;
    static constexpr size_t sz_tiles = (size_t)NTILE * 2 * TP * W;
    static constexpr size_t PSZ = LOWP ? 2 : W;       // bytes of one exchanged p value
    static constexpr size_t sz_pb = 2 * (size_t)F * 2 * 4 * 64 * PSZ;   // [parity][slab][plane][elem][lane]
    static constexpr size_t sz_xb = (size_t)F * 2 * 4 * 64 * W;         // [slab][plane][elem][lane]
    __host__ __device__ static constexpr size_t sz_stage(size_t es) {
        return (((size_t)KP * 16 * es + 15) & ~(size_t)15) + (size_t)KP * 16;
    }
    // The Gram's H: each wave loads its own slab and shares it through LDS
    // (reduced formats and FP32, whose loads outweigh their products), or
    // every wave loads every slab (FP64, bound by its matrix-core rate, where
    // the exchange measured slower)
    static constexpr bool STAGE = FMT != F64;
    // H staged per loaded block: [2 buffers][slab][instruction][re, im, -im][lane] operand fragments
    static constexpr size_t sz_hstage = STAGE ? 2 * (size_t)F * NSUB * 3 * 64 * sizeof(typename Op<FMT, KPLG>::frag) : 0;
    __host__ __device__ static constexpr size_t sz_main(size_t es, bool refresh) {
        size_t a = sz_tiles > sz_hstage ? sz_tiles : sz_hstage, b = sz_pb + (refresh ? sz_xb : 0), c = sz_stage(es);
        return a > b ? (a > c ? a : c) : (b > c ? b : c);
    }
    // L = 8 and 16 keep C and T as 16-wide tiles (block diagonal for L = 8),
    // rows padded to TR words as the tiles of A
    static constexpr int TS = LB >= 8 ? TR : LB;
    static constexpr size_t sz_d = LB ? 2 * W * KP * TS : 0;
    static constexpr size_t sz_t = LB ? 2 * W * KP * TS : 0;
    static constexpr size_t sz_red = 2 * 2 * (size_t)NW * 16 * W;      // [parity][value][wave][column]
    __host__ __device__ static constexpr size_t lds(size_t es, bool split, bool refresh) {
        return sz_main(es, refresh) + sz_d + (split ? 1 : 2) * sz_t + sz_red;
    }
};

// Register budget in waves per SIMD: three (170 registers) where the build
// fits without spilling, two for FP64, K = 128, and the left-form builds with
// the FP64 refresh (which keep a second copy of A and M_d).
template <int KP, int FMT, int LB, bool SPLIT, bool RFR> constexpr int slab_waves() {
    if (FMT == F64 || KP == 128) return 2;
    if (RFR && LB > 0 && !SPLIT) return 2;
    return 3;
}

// index of the upper tile (i, j), i <= j, in row-major order of the upper triangle
__host__ __device__ constexpr int tile_index(int i, int j, int F) { return i * F - i * (i - 1) / 2 + (j - i); }

template <int KP, int FMT, int LB, bool SPLIT, bool RFR, typename IOT>
__global__ __launch_bounds__(64 * (KP / 16)) __attribute__((amdgpu_waves_per_eu(slab_waves<KP, FMT, LB, SPLIT, RFR>())))
void slab_kernel(const FusedParams P) {
    using C = SlabCfg<KP, FMT, LB>;
    using O = typename C::O;
    using OG = typename C::OG;
    using Wt = typename C::Wt;
    using frag = typename O::frag;
    using gfrag = typename OG::frag;
    using acc_t = typename O::acc;
    using gacc_t = typename OG::acc;
    constexpr int NW = C::NW, F = C::F, NT = C::NT, PPW = C::PPW;
    constexpr int KPLG = C::KPLG, NLD = C::NLD, KBG = C::KBG;
    constexpr bool split = (LB > 0) && SPLIT;
    constexpr bool left = (LB > 0) && !SPLIT;
    static_assert(LB < 8 || (SPLIT && FMT != F64), "slab kernel: L = 8 and 16 in the symmetric form, u_W = fp32");
    constexpr uint32_t ES = CxB<IOT>::bytes;
    extern __shared__ __align__(16) unsigned char smem[];

    int64_t ch = blockIdx.x;
    if (P.chan_idx) {
        ch = P.chan_idx[blockIdx.x];
        if (ch < 0 || ch >= P.B) return;
    }
    const int cblk = blockIdx.y;
    const int tid = threadIdx.x;
    // the wave index is uniform over the wave: in a scalar register, its
    // branches (which tiles a wave owns) are scalar branches
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, n = lane & 15;
    const int col = cblk * 16 + n;
    const bool colv = col < P.R;
    const int K = P.K, Nbs = P.Nbs, R = P.R;
    const bool refresh = RFR && P.refresh_every > 0;   // RFR: built with the FP64 refresh
    // Issue priorities among the co-resident workgroups of a CU: the Gram's
    // stream (latency-bound) at 1; the matrix-core throughput work at 0 --
    // the FP64 refresh products, or, without the refresh, the iterations of
    // the reduced and FP32 formats.  (Measured: c3 fp16 with the refresh and
    // FP32 3-4 % faster; FP64 CG slower with it, so FP64 keeps one level.)
    if constexpr (FMT != F64) __builtin_amdgcn_s_setprio(1);

    unsigned char* smain = smem;
    const size_t main_bytes = C::sz_main(ES, refresh);
    Wt* sD = reinterpret_cast<Wt*>(smem + main_bytes);                 // [KP][TS] re, then im
    Wt* sT = reinterpret_cast<Wt*>(smem + main_bytes + C::sz_d);       // T blocks [KP][TS] re, im
    Wt* sM = sT + 2 * KP * (LB ? C::TS : 1);                             // left form: M_d blocks
    Wt* sRed = reinterpret_cast<Wt*>(smem + main_bytes + C::sz_d + (split ? 1 : 2) * C::sz_t);
    __shared__ uint32_t sFlag;
    if (tid == 0) sFlag = 0u;
    uint32_t myflag = 0u;

    const int64_t hoff = ch * (int64_t)Nbs * K, yoff = ch * (int64_t)Nbs * R;
    const Buf bH(static_cast<const char*>(P.H) + hoff * ES, (uint32_t)Nbs * K * ES);
    const Buf bY(static_cast<const char*>(P.Y) + yoff * ES, (uint32_t)Nbs * R * ES);
    const double s2 = P.sigma2[ch];

    // ------------------------------------------------------------ 1. Gram + matched filter
    Wt* sTile = reinterpret_cast<Wt*>(smain);                            // [tile][plane][16 x 16]
    Wt br_[4], bi_[4];                                // b (own slab, rows 4g + i), then b_bar = T b
    {
        gacc_t gAr[PPW], gAi[PPW], gBr, gBi;
#pragma unroll
        for (int s = 0; s < PPW; ++s) { gAr[s] = gacc_t{0, 0, 0, 0}; gAi[s] = gacc_t{0, 0, 0, 0}; }
        gBr = gacc_t{0, 0, 0, 0};
        gBi = gacc_t{0, 0, 0, 0};
        constexpr int NSUB = C::NSUB;
        // Each wave loads only its own slab of H (columns 16 wave + n), rounds
        // it to the operand format and publishes the fragments in LDS; every
        // wave then reads the slabs its tiles need from there.  The next
        // block's loads are issued before this block's products, so one
        // block's memory latency hides behind the other's arithmetic.
        const uint32_t hl = (16 * wave + n < K) ? (uint32_t)(16 * wave + n) * ES : OOB;
        const uint32_t yl = colv ? (uint32_t)col * ES : OOB;
        const uint32_t hrow = (uint32_t)K * ES, yrow = (uint32_t)R * ES;
        // FP64: every wave loads every slab, no exchange
        auto gram_all = [&](auto hcp) {
            uint32_t hlf[F];
#pragma unroll
            for (int f = 0; f < F; ++f) hlf[f] = (16 * f + n < K) ? (uint32_t)(16 * f + n) * ES : OOB;
            for (int a0 = 0; a0 < Nbs; a0 += KBG) {
                Wt xr_[F][NLD], xi_[F][NLD], yr_[NLD], yi_[NLD];
                const uint32_t ab = (uint32_t)(a0 + g * NLD);
#pragma unroll
                for (int j = 0; j < NLD; ++j) {
#pragma unroll
                    for (int f = 0; f < F; ++f)
                        CxB<IOT>::template load<decltype(hcp)::value>(bH, hlf[f] + (ab + j) * hrow, xr_[f][j], xi_[f][j]);
                    CxB<IOT>::load(bY, yl + (ab + j) * yrow, yr_[j], yi_[j]);
                }
#pragma unroll
                for (int u = 0; u < NSUB; ++u) {
                    gfrag Xr[F], Xi[F], nXi[F];
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        Xr[f] = OG::pack(&xr_[f][u * KPLG], 1.f);
                        Xi[f] = OG::pack(&xi_[f][u * KPLG], 1.f);
                        nXi[f] = OG::neg(Xi[f]);
                    }
                    int q = 0;
#pragma unroll
                    for (int f1 = 0; f1 < F; ++f1)
#pragma unroll
                        for (int f2 = f1; f2 < F; ++f2) {
                            if (q % NW == wave) {
                                const int s = q / NW;
                                gAr[s] = OG::mfma(Xr[f1], Xr[f2], gAr[s]);
                                gAr[s] = OG::mfma(Xi[f1], Xi[f2], gAr[s]);
                                gAi[s] = OG::mfma(Xr[f1], Xi[f2], gAi[s]);
                                gAi[s] = OG::mfma(nXi[f1], Xr[f2], gAi[s]);
                            }
                            ++q;
                        }
                    const gfrag Yr = OG::pack(&yr_[u * KPLG], 1.f), Yi = OG::pack(&yi_[u * KPLG], 1.f);
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        if (f == wave) {
                            gBr = OG::mfma(Xr[f], Yr, gBr);
                            gBr = OG::mfma(Xi[f], Yi, gBr);
                            gBi = OG::mfma(Xr[f], Yi, gBi);
                            gBi = OG::mfma(nXi[f], Yr, gBi);
                        }
                    }
                }
            }
        };
        gfrag* sStage = reinterpret_cast<gfrag*>(smain);                 // [2][F][NSUB][3][64]
        auto st_at = [&](int buf, int f, int u, int pl) -> int { return (((buf * F + f) * NSUB + u) * 3 + pl) * 64 + lane; };
        Wt hr[NLD], hi[NLD], yr[NLD], yi[NLD];        // the block in flight
        auto gram_loop = [&](auto hcp) {
            // per-lane parts of the offsets once; the block's and the row's
            // parts are uniform (scalar), one vector add per load
            const uint32_t hbase = hl + (uint32_t)(g * NLD) * hrow, ybase = yl + (uint32_t)(g * NLD) * yrow;
            auto load_block = [&](int a0) {
                const uint32_t ha = (uint32_t)a0 * hrow, ya = (uint32_t)a0 * yrow;
#pragma unroll
                for (int j = 0; j < NLD; ++j) {
                    CxB<IOT>::template load<decltype(hcp)::value>(bH, hbase + (ha + (uint32_t)j * hrow), hr[j], hi[j]);
                    CxB<IOT>::load(bY, ybase + (ya + (uint32_t)j * yrow), yr[j], yi[j]);
                }
            };
            const int nblk = (Nbs + KBG - 1) / KBG;
            load_block(0);
            for (int b = 0; b < nblk; ++b) {
                const int buf = b & 1;
                gfrag Wr_[NSUB], Wi_[NSUB], nWi_[NSUB], Yr[NSUB], Yi[NSUB];
#pragma unroll
                for (int u = 0; u < NSUB; ++u) {
                    Wr_[u] = OG::pack(&hr[u * KPLG], 1.f);
                    Wi_[u] = OG::pack(&hi[u * KPLG], 1.f);
                    nWi_[u] = OG::neg(Wi_[u]);
                    Yr[u] = OG::pack(&yr[u * KPLG], 1.f);
                    Yi[u] = OG::pack(&yi[u * KPLG], 1.f);
                    sStage[st_at(buf, wave, u, 0)] = Wr_[u];
                    sStage[st_at(buf, wave, u, 1)] = Wi_[u];
                    sStage[st_at(buf, wave, u, 2)] = nWi_[u];
                    // Y rounded here, so its registers are free for the next
                    // block's loads (not kept alive beside them)
                    asm volatile("" ::"v"(Yr[u]), "v"(Yi[u]));
                }
                __syncthreads();                      // every slab of this block published
                if (b + 1 < nblk) load_block((b + 1) * KBG);
#pragma unroll
                for (int u = 0; u < NSUB; ++u) {
                    // this wave's tiles q = s NW + wave (slot s), decoded to
                    // their slab pair in scalar registers; operands read
                    // from LDS per tile
#pragma unroll
                    for (int s = 0; s < PPW; ++s) {
                        const int q = s * NW + wave;
                        if (q < C::NTILE) {
                            int f1 = 0;
#pragma unroll
                            for (int i = 1; i < F; ++i)
                                if (q >= tile_index(i, i, F)) f1 = i;
                            const int f2 = f1 + (q - tile_index(f1, f1, F));
                            const gfrag x1r = sStage[st_at(buf, f1, u, 0)], x1i = sStage[st_at(buf, f1, u, 1)];
                            const gfrag nx1i = sStage[st_at(buf, f1, u, 2)];
                            const gfrag x2r = sStage[st_at(buf, f2, u, 0)], x2i = sStage[st_at(buf, f2, u, 1)];
                            gAr[s] = OG::mfma(x1r, x2r, gAr[s]);
                            gAr[s] = OG::mfma(x1i, x2i, gAr[s]);
                            gAi[s] = OG::mfma(x1r, x2i, gAi[s]);
                            gAi[s] = OG::mfma(nx1i, x2r, gAi[s]);
                        }
                    }
                    // matched filter tile of this wave's slab
                    gBr = OG::mfma(Wr_[u], Yr[u], gBr);
                    gBr = OG::mfma(Wi_[u], Yi[u], gBr);
                    gBi = OG::mfma(Wr_[u], Yi[u], gBi);
                    gBi = OG::mfma(nWi_[u], Yr[u], gBi);
                }
            }
            __syncthreads();                          // the stage is read before the tiles overwrite it
        };
        if constexpr (C::STAGE) {
            if (hrow % 128u == 0) gram_loop(std::integral_constant<int, CP_STREAM>{});
            else gram_loop(std::integral_constant<int, 0>{});
        } else {
            if (hrow % 128u == 0) gram_all(std::integral_constant<int, CP_STREAM>{});
            else gram_all(std::integral_constant<int, 0>{});
        }

        // tiles into LDS, row-major per plane (sigma^2 on the diagonal, padding diagonal 1)
        const Wt s2w = (Wt)s2;
        Wt nfa = 0;
        int q = 0;
#pragma unroll
        for (int f1 = 0; f1 < F; ++f1)
#pragma unroll
            for (int f2 = f1; f2 < F; ++f2) {
                if (q % NW == wave) {
                    const int s = q / NW;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int r = OG::crow(g, jj);
                        Wt ar = (Wt)gAr[s][jj], ai = (Wt)gAi[s][jj];
                        if (f1 == f2 && r == n) {
                            ai = 0;
                            ar = (16 * f1 + r < K) ? ar + s2w : (Wt)1;
                        }
                        nfa = fma(ar, (Wt)0, fma(ai, (Wt)0, nfa));
                        sTile[((size_t)q * 2 + 0) * C::TP + r * C::TR + n] = ar;
                        sTile[((size_t)q * 2 + 1) * C::TP + r * C::TR + n] = ai;
                    }
                }
                ++q;
            }
        // the matched filter tile of this wave's slab: the fp32-accumulating
        // shapes hold row 4g + i in element i already; the FP64 shape holds row
        // 4i + g, which lane (i, n) passes back in element g
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if constexpr (FMT == F64) {
                double vr[4], vi[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    vr[e] = __shfl((double)gBr[e], i * 16 + n);
                    vi[e] = __shfl((double)gBi[e], i * 16 + n);
                }
                br_[i] = g == 0 ? vr[0] : g == 1 ? vr[1] : g == 2 ? vr[2] : vr[3];
                bi_[i] = g == 0 ? vi[0] : g == 1 ? vi[1] : g == 2 ? vi[2] : vi[3];
            } else {
                br_[i] = (Wt)gBr[i];
                bi_[i] = (Wt)gBi[i];
            }
            nfa = fma(br_[i], (Wt)0, fma(bi_[i], (Wt)0, nfa));
        }
        if (!__builtin_isfinite(nfa)) myflag |= FLAG_NONFINITE;
    }
    __syncthreads();

    // ------------------------------------------------------------ block-Jacobi setup, L = 8 and 16
    // The Jacobi blocks tile the diagonal 16 x 16 tiles (one block of 16, or
    // two of 8).  Wave w factors the blocks of tile (w, w) -- lane n owns row
    // n % L of block n / L, the factor's columns pass through LDS one step at
    // a time -- and forms their T = C^{-1} by forward substitution, lane n
    // column n % L; T_w, the 16 x 16 block-diagonal tile of T, goes to LDS.
    // Every upper tile is then rewritten in place as T_a A_ab T_b^H, two
    // 16 x 16 x 16 complex products on the fp32 matrix cores, before the
    // waves read their column slabs: A_bar arrives in the layout the
    // iteration uses.  b_bar = T_w b_w likewise.
    if constexpr (LB == 8 || LB == 16) {
        using OF = Op<F32, 1>;
        using f4 = typename OF::acc;
        constexpr int TS = C::TS;                     // row stride of C and T in LDS (a padded tile row)
        Wt* sCr = sD;                                 // C, rows 16 w + r: [KP][TS] re, then im
        Wt* sCi = sD + KP * TS;
        Wt* sTr = sT;                                 // T, the same layout
        Wt* sTi = sT + KP * TS;
        const int rb = 16 * wave;                     // first row of the tile
        const int kb = n / LB, i = n % LB;            // block in the tile, row / column in the block
        const int bb = rb + kb * LB;                  // first row of the block
        const int o0 = kb * LB;                       // first column of the block in the tile
        // the blocks of tile (w, w) are wave w's alone: its lanes exchange the
        // factor's columns through LDS, whose operations a wave issues and
        // completes in order; the fences keep the compiler from moving them
        auto wave_sync = []() {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        Wt tr[LB], ti[LB];
        bool blk_bad = false;
        if (P.T_in) {                                 // a given factor replaces the factorisation
            if (bb < K) {
                const Wt* tin = static_cast<const Wt*>(P.T_in) + ((size_t)ch * K + bb) * LB * 2;
#pragma unroll
                for (int r = 0; r < LB; ++r) { tr[r] = tin[(r * LB + i) * 2]; ti[r] = tin[(r * LB + i) * 2 + 1]; }
            } else {                                  // padding block: the identity
#pragma unroll
                for (int r = 0; r < LB; ++r) { tr[r] = r == i ? (Wt)1 : (Wt)0; ti[r] = 0; }
            }
        } else {
            const int qd = tile_index(wave, wave, F);
            Wt ar[LB], ai[LB];
#pragma unroll
            for (int c = 0; c < LB; ++c) {
                ar[c] = sTile[((size_t)qd * 2 + 0) * C::TP + n * C::TR + o0 + c];
                ai[c] = sTile[((size_t)qd * 2 + 1) * C::TP + n * C::TR + o0 + c];
            }
            Wt diag = 0;                              // a_ii, for the not-PD fallback
#pragma unroll
            for (int c = 0; c < LB; ++c)
                if (c == i) diag = ar[c];
            bool bad = false;
#pragma unroll
            for (int j = 0; j < LB; ++j) {
                if (i == j) {
                    Wt d = ar[j];
                    if (!(d > 0) || !__builtin_isfinite(d)) { bad = true; d = 1; }
                    const Wt l = sqrt(d);
                    if (g == 0) { sCr[(bb + j) * TS + o0 + j] = l; sCi[(bb + j) * TS + o0 + j] = (Wt)1 / l; }
                }
                wave_sync();
                const Wt inv = sCi[(bb + j) * TS + o0 + j];
                const Wt lr = ar[j] * inv, li = ai[j] * inv;
                if (i > j && g == 0) { sCr[(bb + i) * TS + o0 + j] = lr; sCi[(bb + i) * TS + o0 + j] = li; }
                wave_sync();
                if (i > j) {
#pragma unroll
                    for (int k = j + 1; k < LB; ++k) {   // a_ik -= l_ij conj(l_kj), needed for k <= i
                        const Wt kr = sCr[(bb + k) * TS + o0 + j], ki = sCi[(bb + k) * TS + o0 + j];
                        ar[k] = fma(-lr, kr, fma(-li, ki, ar[k]));
                        ai[k] = fma(-li, kr, fma(lr, ki, ai[k]));
                    }
                }
            }
            // the lanes of one block: lane groups x the block's 16 / (16 / L) lanes
            const uint64_t grp = (LB == 16) ? ~0ull : 0x00FF00FF00FF00FFull << (kb * LB);
            blk_bad = (__ballot(bad) & grp) != 0;
            // column i of T = C^{-1}: C t = e_i by forward substitution, a
            // column of C at a time (the imaginary diagonal slot holds 1 / c_mm)
#pragma unroll
            for (int r = 0; r < LB; ++r) { tr[r] = r == i ? (Wt)1 : (Wt)0; ti[r] = 0; }
            int cm = bb * TS + o0;                    // offset of the block's C
#pragma unroll
            for (int m = 0; m < LB; ++m) {
                const Wt inv_mm = sCi[cm + m * TS + m];
                tr[m] = tr[m] * inv_mm;
                ti[m] = ti[m] * inv_mm;
                // the column's loads wait for t_m: an offset that depends on it
                // keeps them from all being issued ahead into registers
                asm("" : "+v"(cm) : "v"(tr[m]), "v"(ti[m]));
#pragma unroll
                for (int r = m + 1; r < LB; ++r) {   // t_r -= c_rm t_m
                    const Wt cr_ = sCr[cm + r * TS + m], ci_ = sCi[cm + r * TS + m];
                    tr[r] = fma(-cr_, tr[m], fma(ci_, ti[m], tr[r]));
                    ti[r] = fma(-cr_, ti[m], fma(-ci_, tr[m], ti[r]));
                }
            }
            if (blk_bad) {
                // not positive definite: T = diag(a_ii)^{-1/2}, so M_d = diag(a_ii)^{-1}
#pragma unroll
                for (int r = 0; r < LB; ++r) {
                    tr[r] = 0; ti[r] = 0;
                    if (r == i) tr[r] = (diag > 0 && __builtin_isfinite(diag)) ? (Wt)1 / sqrt(diag) : (Wt)1;
                }
                myflag |= FLAG_BLOCK_NOT_PD;
            }
        }
        if (g == 0) {
            // column n of the tile of T: the block's column, zeros beside it
#pragma unroll
            for (int r = 0; r < LB; ++r) { sTr[(bb + r) * TS + n] = tr[r]; sTi[(bb + r) * TS + n] = ti[r]; }
            if constexpr (LB < 16) {
#pragma unroll
                for (int r = 0; r < LB; ++r) {
                    const int orow = rb + (kb ^ 1) * LB + r;
                    sTr[orow * TS + n] = 0;
                    sTi[orow * TS + n] = 0;
                }
            }
            if (P.T_out && cblk == 0 && bb < K) {     // column i of this block of T
                Wt* tout = static_cast<Wt*>(P.T_out) + ((size_t)ch * K + bb) * LB * 2;
#pragma unroll
                for (int r = 0; r < LB; ++r) { tout[(r * LB + i) * 2] = tr[r]; tout[(r * LB + i) * 2 + 1] = ti[r]; }
            }
        }
        __syncthreads();                              // every block of T in LDS
        // the tiles this wave formed in the Gram, in place
#pragma unroll
        for (int s = 0; s < PPW; ++s) {
            const int q = s * NW + wave;
            if (q < C::NTILE) {
                int a = 0;
#pragma unroll
                for (int f = 1; f < F; ++f)
                    if (q >= tile_index(f, f, F)) a = f;
                const int b = a + (q - tile_index(a, a, F));
                Wt* tre = sTile + ((size_t)q * 2 + 0) * C::TP;
                Wt* tim = sTile + ((size_t)q * 2 + 1) * C::TP;
                // X = A_ab T_b^H: operand lane (g', n') holds A_ab[n'][4 e + g'] and
                // conj(T_b[n'][4 e + g']) for contraction step e
                f4 Xr = f4{0, 0, 0, 0}, Xi = f4{0, 0, 0, 0};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int j = 4 * e + g;
                    const Wt a_r = tre[n * C::TR + j], a_i = tim[n * C::TR + j];
                    const Wt t_r = sTr[(16 * b + n) * TS + j], t_i = sTi[(16 * b + n) * TS + j];
                    Xr = OF::mfma(a_r, t_r, Xr);
                    Xr = OF::mfma(a_i, t_i, Xr);
                    Xi = OF::mfma(a_i, t_r, Xi);
                    Xi = OF::mfma(-a_r, t_i, Xi);
                }
                // A_bar_ab = T_a X: X[4 g' + e][n'] is element e of the lane's own
                // output, T_a[n'][4 g' + e] the matching operand
                f4 Ur = f4{0, 0, 0, 0}, Ui = f4{0, 0, 0, 0};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 4 * g + e;
                    const Wt t_r = sTr[(16 * a + n) * TS + r], t_i = sTi[(16 * a + n) * TS + r];
                    Ur = OF::mfma(t_r, Xr[e], Ur);
                    Ur = OF::mfma(-t_i, Xi[e], Ur);
                    Ui = OF::mfma(t_r, Xi[e], Ui);
                    Ui = OF::mfma(t_i, Xr[e], Ui);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    tre[(4 * g + e) * C::TR + n] = Ur[e];
                    tim[(4 * g + e) * C::TR + n] = Ui[e];
                }
            }
        }
        // b_bar = T_w b_w
        {
            f4 Ur = f4{0, 0, 0, 0}, Ui = f4{0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 4 * g + e;
                const Wt t_r = sTr[(rb + n) * TS + r], t_i = sTi[(rb + n) * TS + r];
                Ur = OF::mfma(t_r, br_[e], Ur);
                Ur = OF::mfma(-t_i, bi_[e], Ur);
                Ui = OF::mfma(t_r, bi_[e], Ui);
                Ui = OF::mfma(t_i, br_[e], Ui);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) { br_[e] = Ur[e]; bi_[e] = Ui[e]; }
        }
        __syncthreads();                              // every tile rewritten
        // the diagonal tile of this wave exactly Hermitian: the lower triangle
        // the conjugate of the upper one, the diagonal real
        {
            const int qd = tile_index(wave, wave, F);
            Wt* tre = sTile + ((size_t)qd * 2 + 0) * C::TP;
            Wt* tim = sTile + ((size_t)qd * 2 + 1) * C::TP;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 4 * g + e;
                if (r > n) {
                    tre[r * C::TR + n] = tre[n * C::TR + r];
                    tim[r * C::TR + n] = -tim[n * C::TR + r];
                } else if (r == n) {
                    tim[r * C::TR + n] = 0;
                }
            }
        }
        __syncthreads();
    }

    // ------------------------------------------------------------ column slab of A, own slab of b
    // Acol[f][i]: A[16f + 4g + i][16 wave + n]; AcP[f][i]: the same for column
    // 16 wave + rho(n) (the FP64 operand layout, for FP64 A p and the refresh)
    constexpr bool NEED_STD = (FMT != F64);
    constexpr bool NEED_PERM = (FMT == F64);          // (reduced formats keep a permuted copy for the refresh)
    Wt Acr[F][4], Aci[F][4];                          // standard (reduced formats) or permuted (FP64)
    Wt Apr[RFR && !NEED_PERM ? F : 1][4], Api[RFR && !NEED_PERM ? F : 1][4];   // permuted copy for the FP64 refresh
    auto a_at = [&](int row, int c, Wt& re, Wt& im) {   // A[row][c] from the tiles in LDS
        const int fr = row >> 4, fc = c >> 4, rr = row & 15, cc = c & 15;
        if (fr <= fc) {
            const int q = tile_index(fr, fc, F);
            re = sTile[((size_t)q * 2 + 0) * C::TP + rr * C::TR + cc];
            im = sTile[((size_t)q * 2 + 1) * C::TP + rr * C::TR + cc];
        } else {
            const int q = tile_index(fc, fr, F);
            re = sTile[((size_t)q * 2 + 0) * C::TP + cc * C::TR + rr];
            im = -sTile[((size_t)q * 2 + 1) * C::TP + cc * C::TR + rr];
        }
    };
    const int cstd = 16 * wave + n, cperm = 16 * wave + rho16(n);
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * f + 4 * g + i;
            a_at(row, NEED_STD ? cstd : cperm, Acr[f][i], Aci[f][i]);
            if constexpr (RFR && !NEED_PERM) a_at(row, cperm, Apr[f][i], Api[f][i]);
        }
    if constexpr (LB == 4) {
        // diagonal blocks of this slab (standard columns: tile (wave, wave) in Acr / Aci
        // for the reduced formats; FP64 holds permuted columns, so read them from LDS)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * wave + 4 * g + i, c = 16 * wave + n;
            if (row / LB == c / LB) {
                Wt re, im;
                a_at(row, c, re, im);
                sD[row * LB + c % LB] = re;
                sD[KP * LB + row * LB + c % LB] = im;
            }
        }
    }
    __syncthreads();                                  // every wave has its slab; the tile region is free

    // ------------------------------------------------------------ 2. block-Jacobi setup (L = 4)
    Wt Mr[LB ? 4 : 1][LB ? 4 : 1], Mi[LB ? 4 : 1][LB ? 4 : 1];   // this lane's block of M_d (left form)
    if constexpr (LB == 4) {
        {
            const bool act = tid < KP;
            const int t = act ? tid : 0;
            const int i = t % LB, cb = t - i;
            Wt tr[LB], ti[LB];
            bool blk_bad = false;
            if (P.T_in) {                             // a given factor replaces the factorisation
                if (act && cb < K) {
                    const Wt* tin = static_cast<const Wt*>(P.T_in) + ((size_t)ch * K + cb) * LB * 2;
#pragma unroll
                    for (int r = 0; r < LB; ++r) { tr[r] = tin[(r * LB + i) * 2]; ti[r] = tin[(r * LB + i) * 2 + 1]; }
                } else {                              // padding blocks: the identity
#pragma unroll
                    for (int r = 0; r < LB; ++r) { tr[r] = r == i ? (Wt)1 : (Wt)0; ti[r] = 0; }
                }
            } else {
                Wt cr[LB][LB], ci[LB][LB];
#pragma unroll
                for (int r = 0; r < LB; ++r)
#pragma unroll
                    for (int c = 0; c <= r; ++c) { cr[r][c] = sD[(cb + r) * LB + c]; ci[r][c] = sD[KP * LB + (cb + r) * LB + c]; }
                Wt diag = 0;
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
                            cr[r][c] = fma(-cr[r][j], cr[c][j], fma(-ci[r][j], ci[c][j], cr[r][c]));
                            ci[r][c] = fma(-ci[r][j], cr[c][j], fma(cr[r][j], ci[c][j], ci[r][c]));
                        }
                }
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
                if (blk_bad) {
#pragma unroll
                    for (int r = 0; r < LB; ++r) {
                        tr[r] = 0; ti[r] = 0;
                        if (r == i) tr[r] = (diag > 0 && __builtin_isfinite(diag)) ? (Wt)1 / sqrt(diag) : (Wt)1;
                    }
                }
            }
            if (act) {
#pragma unroll
                for (int r = 0; r < LB; ++r) {                   // column i of T
                    sT[(cb + r) * LB + i] = tr[r];
                    sT[KP * LB + (cb + r) * LB + i] = ti[r];
                }
                if (blk_bad && i == 0) myflag |= FLAG_BLOCK_NOT_PD;
                if (P.T_out && cblk == 0 && cb < K) {  // column i of this block of T
                    Wt* tout = static_cast<Wt*>(P.T_out) + ((size_t)ch * K + cb) * LB * 2;
#pragma unroll
                    for (int r = 0; r < LB; ++r) { tout[(r * LB + i) * 2] = tr[r]; tout[(r * LB + i) * 2 + 1] = ti[r]; }
                }
            }
            if constexpr (left) {
                __syncthreads();
                if (act) {
#pragma unroll
                    for (int j = 0; j < LB; ++j) {                // M = T^H T: row i
                        Wt mr = 0, mi = 0;
#pragma unroll
                        for (int m = 0; m < LB; ++m) {
                            const Wt b_r = sT[(cb + m) * LB + j], b_i = sT[KP * LB + (cb + m) * LB + j];
                            mr = fma(tr[m], b_r, fma(ti[m], b_i, mr));
                            mi = fma(tr[m], b_i, fma(-ti[m], b_r, mi));
                        }
                        sM[(cb + i) * LB + j] = mr;
                        sM[KP * LB + (cb + i) * LB + j] = mi;
                    }
                }
            }
        }
        __syncthreads();
        // this lane's blocks: rows 16 wave + 4 g + (0..3) form block 4 wave + g
        const int rb = 16 * wave + 4 * g;
        if constexpr (left) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    Mr[r][j] = sM[(rb + r) * LB + j];
                    Mi[r][j] = sM[KP * LB + (rb + r) * LB + j];
                }
        }
        if constexpr (split) {
            // A <- T A T^H.  Rows: tile f, lane group g are rows of block 4f + g,
            // mixed lane-locally by that block of T.  Columns: column 16 wave + n
            // is column n % 4 of block 4 wave + n / 4, whose other columns sit in
            // the three neighbouring lanes of the quad.
            auto rows_T = [&](Wt (&vr)[F][4], Wt (&vi)[F][4]) {
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const int rbf = 16 * f + 4 * g;
                    Wt t_r[4][4], t_i[4][4];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int j = 0; j <= r; ++j) { t_r[r][j] = sT[(rbf + r) * LB + j]; t_i[r][j] = sT[KP * LB + (rbf + r) * LB + j]; }
                    Wt ur[4], ui[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        Wt sr = 0, si = 0;
#pragma unroll
                        for (int j = 0; j <= r; ++j) {
                            sr = fma(t_r[r][j], vr[f][j], fma(-t_i[r][j], vi[f][j], sr));
                            si = fma(t_r[r][j], vi[f][j], fma(t_i[r][j], vr[f][j], si));
                        }
                        ur[r] = sr; ui[r] = si;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) { vr[f][r] = ur[r]; vi[f][r] = ui[r]; }
                }
            };
            // columns of the standard layout: lane n holds column n
            auto cols_TH = [&](Wt (&vr)[F][4], Wt (&vi)[F][4], int cbase) {
                // T block of column block cbase / 4 (T[cc][j], j <= cc) for this lane's column cc = n % 4
                const int cc = n & 3;
                Wt t_r[4], t_i[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    t_r[j] = sT[(cbase + cc) * LB + j];
                    t_i[j] = sT[KP * LB + (cbase + cc) * LB + j];
                }
#pragma unroll
                for (int f = 0; f < F; ++f)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        Wt sr = 0, si = 0;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {      // += W[.][j] conj(T[cc][j]), T[cc][j] = 0 for j > cc
                            const Wt wr = quad_bcast(vr[f][i], j), wi = quad_bcast(vi[f][i], j);
                            sr = fma(wr, t_r[j], fma(wi, t_i[j], sr));
                            si = fma(wi, t_r[j], fma(-wr, t_i[j], si));
                        }
                        vr[f][i] = sr; vi[f][i] = si;
                    }
            };
            if constexpr (FMT == F64) {
                // permuted columns in registers: transform the standard ones, then permute
                Wt sr_[F][4], si_[F][4];
#pragma unroll
                for (int f = 0; f < F; ++f)
#pragma unroll
                    for (int i = 0; i < 4; ++i) a_at(16 * f + 4 * g + i, cstd, sr_[f][i], si_[f][i]);
                rows_T(sr_, si_);
                cols_TH(sr_, si_, 16 * wave + (n & ~3));
#pragma unroll
                for (int f = 0; f < F; ++f)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        Acr[f][i] = __shfl(sr_[f][i], g * 16 + rho16(n));
                        Aci[f][i] = __shfl(si_[f][i], g * 16 + rho16(n));
                    }
            } else {
                rows_T(Acr, Aci);
                cols_TH(Acr, Aci, 16 * wave + (n & ~3));
                if constexpr (RFR) {
#pragma unroll
                    for (int f = 0; f < F; ++f)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            Apr[f][i] = __shfl(Acr[f][i], g * 16 + rho16(n));
                            Api[f][i] = __shfl(Aci[f][i], g * 16 + rho16(n));
                        }
                }
            }
            // b_bar = T b (rows of block 4 wave + g)
            Wt ur[4], ui[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Wt sr = 0, si = 0;
#pragma unroll
                for (int j = 0; j <= r; ++j) {
                    const Wt t_r = sT[(rb + r) * LB + j], t_i = sT[KP * LB + (rb + r) * LB + j];
                    sr = fma(t_r, br_[j], fma(-t_i, bi_[j], sr));
                    si = fma(t_r, bi_[j], fma(t_i, br_[j], si));
                }
                ur[r] = sr; ui[r] = si;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) { br_[r] = ur[r]; bi_[r] = ui[r]; }
        }
    }

    // ------------------------------------------------------------ A operand in registers
    // A p for rows of slab `wave` contracts row slab `wave` of A, the conjugate
    // of the column slab held: A[16 wave + n'][16 f + 4 g' + k] = conj(Acol[f][k])
    // of lane (g', n').  Re(W) = Ar pr + Ai pi, Im(W) = Ar pi - Ai pr (Ai = Im Acol).
    constexpr int NCH = C::LOWP ? F / 2 : F * 4;      // contraction chunks
    frag afr[NCH][2];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if constexpr (C::LOWP) {
            Wt vr[8], vi[8];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                vr[k] = Acr[2 * c][k]; vi[k] = Aci[2 * c][k];
                vr[4 + k] = Acr[2 * c + 1][k]; vi[4 + k] = Aci[2 * c + 1][k];
            }
            afr[c][0] = O::pack(vr, 1.f);
            afr[c][1] = O::pack(vi, 1.f);
        } else {
            afr[c][0] = (frag)Acr[c / 4][c % 4];
            afr[c][1] = (frag)Aci[c / 4][c % 4];
        }
    }
    // Im(W) takes -Ai pr: a negated copy of the imaginary operand, so that no
    // sign is flipped per iteration (the products are the same)
    frag afn[FMT == F64 ? 1 : NCH];
    if constexpr (FMT != F64) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if constexpr (C::LOWP) afn[c] = O::neg(afr[c][1]);
            else afn[c] = -afr[c][1];
        }
    }

    // ------------------------------------------------------------ 3. (P)CG
    unsigned char* sPB = smain;          // p exchange: [2][F][2][4][64] (u_W), [2][F/2][2][64][8 halves] (reduced)
    Wt* sXB = reinterpret_cast<Wt*>(smain + C::sz_pb);                // x exchange [F][2][4][64]
    auto pb_at = [&](int par, int s, int pl, int e, int ln) -> size_t {
        return ((((size_t)par * F + s) * 2 + pl) * 4 + e) * 64 + ln;
    };
    // publish this wave's slab of p in the operand format (reduced) or u_W
    auto publish_p = [&](int par, const Wt* pr, const Wt* pi) {
        if constexpr (C::LOWP) {
            uint32_t* d = reinterpret_cast<uint32_t*>(sPB);
            // four halves of a plane as two words, beside those of the other
            // slab of the same contraction chunk: [par][chunk][plane][lane][slab & 1][2 words]
            const size_t o = (((size_t)par * NCH + (wave >> 1)) * 2) * 64 * 4 + (wave & 1) * 2;
            uint32_t w0, w1, v0, v1;
            if constexpr (FMT == F16) {
                w0 = f16x2_bits(pr[0], pr[1]); w1 = f16x2_bits(pr[2], pr[3]);
                v0 = f16x2_bits(pi[0], pi[1]); v1 = f16x2_bits(pi[2], pi[3]);
            } else {
                w0 = bf16x2_bits(pr[0], pr[1]); w1 = bf16x2_bits(pr[2], pr[3]);
                v0 = bf16x2_bits(pi[0], pi[1]); v1 = bf16x2_bits(pi[2], pi[3]);
            }
            *reinterpret_cast<u32x2*>(d + o + (size_t)lane * 4) = u32x2{w0, w1};
            *reinterpret_cast<u32x2*>(d + o + 256 + (size_t)lane * 4) = u32x2{v0, v1};
        } else {
            Wt* d = reinterpret_cast<Wt*>(sPB);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                d[pb_at(par, wave, 0, e, lane)] = pr[e];
                d[pb_at(par, wave, 1, e, lane)] = pi[e];
            }
        }
    };
    // B operand of chunk c, plane pl, from parity par
    auto b_op = [&](int par, int c, int pl) -> frag {
        if constexpr (C::LOWP) {
            // the parity's part of the offset once, the chunk's and plane's
            // parts as constants
            const uint32_t* d = reinterpret_cast<const uint32_t*>(sPB) + (size_t)par * NCH * 2 * 64 * 4 + lane * 4;
            return *reinterpret_cast<const frag*>(d + (size_t)(c * 2 + pl) * 64 * 4);
        } else {
            const Wt* d = reinterpret_cast<const Wt*>(sPB);
            return (frag)d[pb_at(par, c / 4, pl, c % 4, lane)];
        }
    };
    // sums of a per-lane value over the column (lane groups, then waves in
    // order), two values at once; slot k of parity par
    auto reduce2 = [&](int par, Wt& v0, Wt& v1, int cnt) {
        v0 = col_sum(v0);
        if (cnt > 1) v1 = col_sum(v1);
        Wt* red = sRed + (size_t)par * 2 * NW * 16;
        if (g == 0) {
            red[(0 * NW + wave) * 16 + n] = v0;
            if (cnt > 1) red[(1 * NW + wave) * 16 + n] = v1;
        }
        __syncthreads();
        Wt a = red[(0 * NW + 0) * 16 + n], b = cnt > 1 ? red[(1 * NW + 0) * 16 + n] : (Wt)0;
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            a = a + red[(0 * NW + w) * 16 + n];
            if (cnt > 1) b = b + red[(1 * NW + w) * 16 + n];
        }
        v0 = a;
        v1 = b;
    };

    Wt xr[4], xi[4], rr[4], ri[4], pr[4], pi[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) { xr[e] = 0; xi[e] = 0; rr[e] = br_[e]; ri[e] = bi_[e]; }
    auto apply_M = [&](const Wt* ur, const Wt* ui, Wt* zr, Wt* zi) {
        if constexpr (left) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Wt sr = 0, si = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    sr = fma(Mr[r][j], ur[j], fma(-Mi[r][j], ui[j], sr));
                    si = fma(Mr[r][j], ui[j], fma(Mi[r][j], ur[j], si));
                }
                zr[r] = sr; zi[r] = si;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) { zr[e] = ur[e]; zi[e] = ui[e]; }
        }
    };
    apply_M(rr, ri, pr, pi);                          // p0 = M r0 (Alg. 3) or r0
    int par = 0;
    Wt rho_cur;
    {
        Wt v0 = 0, v1 = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) { v0 = fma(rr[e], pr[e], v0); v0 = fma(ri[e], pi[e], v0); }
        reduce2(par, v0, v1, 1);
        rho_cur = v0;
    }
    publish_p(par, pr, pi);
    __syncthreads();
    // flags so far, wave-uniform
    uint32_t wflag = 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        if (__ballot((myflag >> b) & 1u) != 0) wflag |= 1u << b;
    myflag = 0u;
    bool live = true, broken = false;
    if constexpr (FMT != F64)
        if (!refresh) __builtin_amdgcn_s_setprio(0);
    for (int it = 1; it <= P.iters; ++it) {
        // ---- varpi = A p   [u_MV]
        Wt wr[4], wi[4];
        if constexpr (FMT == F64) {
            // FP64: three real products per complex one, as in the refresh
            acc_t P1 = acc_t{0, 0, 0, 0}, P2 = acc_t{0, 0, 0, 0}, P3 = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const frag b_r = b_op(par, c, 0), b_i = b_op(par, c, 1);
                // (the difference is formed here, not kept: a copy that
                // depends on the iteration cannot be hoisted out of the loop
                // into registers, and, not volatile, does not order the loads)
                double a_r = afr[c][0];
                asm("" : "+v"(a_r) : "s"(it));
                P1 = O::mfma(afr[c][0], b_r, P1);
                P2 = O::mfma(afr[c][1], b_i, P2);
                P3 = O::mfma(a_r - afr[c][1], b_r + b_i, P3);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) { wr[e] = P1[e] + P2[e]; wi[e] = (P3[e] - P1[e]) + P2[e]; }
        } else {
            acc_t Wr = acc_t{0, 0, 0, 0}, Wi = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const frag b_r = b_op(par, c, 0), b_i = b_op(par, c, 1);
                Wr = O::mfma(afr[c][0], b_r, Wr);
                Wr = O::mfma(afr[c][1], b_i, Wr);
                Wi = O::mfma(afr[c][0], b_i, Wi);
                Wi = O::mfma(afn[c], b_r, Wi);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) { wr[e] = (Wt)Wr[e]; wi[e] = (Wt)Wi[e]; }
        }
        // ---- phi = p^H varpi, rho_{i-1} (Alg. 3 as printed)  [u_IP]
        const bool need_rp = left && (P.variant == 0);
        Wt v0 = 0, v1 = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) { v0 = fma(pr[e], wr[e], v0); v0 = fma(pi[e], wi[e], v0); }
        if (need_rp) {
#pragma unroll
            for (int e = 0; e < 4; ++e) { v1 = fma(rr[e], pr[e], v1); v1 = fma(ri[e], pi[e], v1); }
        }
        reduce2(par, v0, v1, need_rp ? 2 : 1);
        const Wt ph = v0;
        const Wt rho_prev = need_rp ? v1 : rho_cur;
        // ---- guard, alpha, x and r  [u_W]
        const bool ok = live && __builtin_isfinite(ph) && __builtin_isfinite(rho_prev) && ph > 0 && rho_prev > 0;
        if (live && !ok && colv) broken = true;
        live = ok;
        Wt alpha_rec = 0, beta_rec = 0;
        if (live) {
            const Wt alpha = rho_prev / ph;
            alpha_rec = alpha;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                xr[e] = fma(alpha, pr[e], xr[e]);
                xi[e] = fma(alpha, pi[e], xi[e]);
                rr[e] = fma(-alpha, wr[e], rr[e]);
                ri[e] = fma(-alpha, wi[e], ri[e]);
            }
        }
        // ---- FP64 residual refresh r = b - A x on the stored u_W matrix
        if (RFR && refresh && it % P.refresh_every == 0 && it < P.iters) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sXB[(((size_t)wave * 2 + 0) * 4 + e) * 64 + lane] = xr[e];
                sXB[(((size_t)wave * 2 + 1) * 4 + e) * 64 + lane] = xi[e];
            }
            __syncthreads();
            // the refresh's FP64 products are throughput work: its waves issue
            // at the lowest priority, so that the latency-bound phases of
            // co-resident workgroups (the Gram's loads and products, the
            // iterations' chains) take the matrix cores between them
            __builtin_amdgcn_s_setprio(0);
            // three real products per complex one: with the row of A as
            // a_r - i a_i, Re = P1 + P2 and Im = P3 + (P2 - P1) for P1 = a_r x_r,
            // P2 = a_i x_i, P3 = (a_r - a_i)(x_r + x_i); two passes, so that
            // no more than two accumulators are live at once
            auto a_of = [&](int c, double& a_r, double& a_i) {
                const int f = c / 4, k = c % 4;
                if constexpr (NEED_PERM) { a_r = (double)Acr[f][k]; a_i = (double)Aci[f][k]; }
                else {
                    // widened here, from copies that depend on the iteration,
                    // so that A is held in u_W and not as hoisted FP64 copies
                    Wt ar = Apr[RFR ? f : 0][k], ai = Api[RFR ? f : 0][k];
                    asm("" : "+v"(ar), "+v"(ai) : "s"(it));
                    a_r = (double)ar; a_i = (double)ai;
                }
            };
            auto x_of = [&](int c, int pl) -> double {
                return (double)sXB[(((size_t)(c / 4) * 2 + pl) * 4 + c % 4) * 64 + lane];
            };
            f64x4 P1 = f64x4{0, 0, 0, 0}, P2 = f64x4{0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < F * 4; ++c) {
                double a_r, a_i;
                a_of(c, a_r, a_i);
                P1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r, x_of(c, 0), P1, 0, 0, 0);
                P2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i, x_of(c, 1), P2, 0, 0, 0);
            }
            f64x4 D;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                D[e] = P2[e] - P1[e];
                Wt be = br_[e];
                asm("" : "+v"(be) : "s"(it));         // converted here, not hoisted out of the loop
                if (live) rr[e] = (Wt)((double)be - (P1[e] + P2[e]));
            }
            f64x4 P3 = f64x4{0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < F * 4; ++c) {
                double a_r, a_i;
                a_of(c, a_r, a_i);
                P3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r - a_i, x_of(c, 0) + x_of(c, 1), P3, 0, 0, 0);
            }
            if (live) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    Wt be = bi_[e];
                    asm("" : "+v"(be) : "s"(it));
                    ri[e] = (Wt)((double)be - (P3[e] + D[e]));
                }
            }
            // (the x exchange is next written at the next refresh, at least
            // three barriers later, so no barrier is needed after the reads)
            __builtin_amdgcn_s_setprio(1);
        }
        // ---- z = M r (left form) or r, rho_i, beta, p
        Wt zr[4], zi[4];
        apply_M(rr, ri, zr, zi);
        v0 = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) { v0 = fma(rr[e], zr[e], v0); v0 = fma(ri[e], zi[e], v0); }
        reduce2(par ^ 1, v0, v1, 1);
        const Wt rho_new = v0;
        if (live) {
            const Wt beta = rho_new / rho_prev;
            beta_rec = beta;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                pr[e] = fma(beta, pr[e], zr[e]);
                pi[e] = fma(beta, pi[e], zi[e]);
            }
        }
        rho_cur = rho_new;
        if (P.ab_hist && g == 0 && wave == 0 && colv && col < KAPPA_COLS) {
            const int nrec = R < KAPPA_COLS ? R : KAPPA_COLS;
            float* h = P.ab_hist + (((int64_t)blockIdx.x * nrec + col) * P.iters + (it - 1)) * 2;
            h[0] = (float)alpha_rec;
            h[1] = (float)beta_rec;
        }
        par ^= 1;
        publish_p(par, pr, pi);
        __syncthreads();
    }
    if (broken) myflag |= FLAG_BREAKDOWN;

    // ------------------------------------------------------------ 4. back-transform, slicer, stores
    if constexpr (split && (LB == 8 || LB == 16)) {   // x = T_w^H x_bar on the matrix cores
        using OF = Op<F32, 1>;
        using f4 = typename OF::acc;
        constexpr int TS = C::TS;
        const Wt* sTr = sT;
        const Wt* sTi = sT + KP * TS;
        const int rb = 16 * wave;
        // x[r] = sum_j conj(T_w[j][r]) x_bar[j]: operand lane (g', n') holds
        // conj(T_w[4 g' + e][n']) for contraction element e, x_bar[4 g' + e] its own
        f4 Ur = f4{0, 0, 0, 0}, Ui = f4{0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const Wt t_r = sTr[(rb + 4 * g + e) * TS + n], t_i = sTi[(rb + 4 * g + e) * TS + n];
            Ur = OF::mfma(t_r, xr[e], Ur);
            Ur = OF::mfma(t_i, xi[e], Ur);
            Ui = OF::mfma(t_r, xi[e], Ui);
            Ui = OF::mfma(-t_i, xr[e], Ui);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) { xr[e] = Ur[e]; xi[e] = Ui[e]; }
    } else if constexpr (split) {                     // x = T^H x_bar (rows of block 4 wave + g)
        const int rb = 16 * wave + 4 * g;
        Wt ur[4], ui[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Wt sr = 0, si = 0;
#pragma unroll
            for (int j = r; j < 4; ++j) {             // += conj(T[j][r]) x_j
                const Wt t_r = sT[(rb + j) * LB + r], t_i = sT[KP * LB + (rb + j) * LB + r];
                sr = fma(t_r, xr[j], fma(t_i, xi[j], sr));
                si = fma(t_r, xi[j], fma(-t_i, xr[j], si));
            }
            ur[r] = sr; ui[r] = si;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) { xr[r] = ur[r]; xi[r] = ui[r]; }
    }
    {
        const Wt nu = (Wt)P.nu, mm = (Wt)P.m;
        const bool stage = R <= 16;
        unsigned char* so_x = smain;
        unsigned char* so_l = so_x + (((size_t)K * R * ES + 15) & ~(size_t)15);
        if (stage) __syncthreads();                     // every wave is done with the exchange region
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 16 * wave + 4 * g + e;
            const uint8_t lab = slice_label<Wt>(xr[e], xi[e], nu, mm, P.m, P.bits);
            if (stage) {
                if (colv && row < K) {
                    const int o = row * R + col;
                    IOT* px = reinterpret_cast<IOT*>(so_x + (size_t)o * ES);
                    px[0] = (IOT)xr[e];
                    px[1] = (IOT)xi[e];
                    so_l[o] = lab;
                }
            } else {
                const Buf bXo(static_cast<char*>(P.xhat) + (int64_t)ch * K * R * ES, (uint32_t)K * R * ES);
                const Buf bLo(P.labels + (int64_t)ch * K * R, (uint32_t)K * R);
                const uint32_t o = (uint32_t)row * R;
                CxB<IOT>::store(bXo, (colv && row < K ? (uint32_t)col * ES : OOB) + o * ES, xr[e], xi[e]);
                store_u8(bLo, (colv && row < K ? (uint32_t)col : OOB) + o, lab);
            }
        }
        if (stage) {
            __syncthreads();
            const Buf bXo(static_cast<char*>(P.xhat) + (int64_t)ch * K * R * ES, (uint32_t)K * R * ES);
            const Buf bLo(P.labels + (int64_t)ch * K * R, (uint32_t)K * R);
            const uint32_t nx = (uint32_t)K * R * ES, nl = (uint32_t)K * R;
            for (uint32_t i = tid * 16u; i + 16u <= nx; i += NT * 16u)
                store_b128<CP_STREAM>(bXo, i, *reinterpret_cast<const u32x4v*>(so_x + i));
            if ((nx & 15u) && tid == 0) {
                const uint32_t i = nx & ~15u;
                store_b64<CP_STREAM>(bXo, i, *reinterpret_cast<const u32x2v*>(so_x + i));
            }
            for (uint32_t i = tid * 16u; i + 16u <= nl; i += NT * 16u)
                store_b128<0>(bLo, i, *reinterpret_cast<const u32x4v*>(so_l + i));
            for (uint32_t i = (nl & ~15u) + tid; i < nl; i += NT) store_u8(bLo, i, so_l[i]);
        }
    }
    myflag |= wflag;
    if (myflag) atomicOr(&sFlag, myflag);
    __syncthreads();
    if (tid == 0 && P.flags) {
        if (P.R <= 16) P.flags[ch] = sFlag;
        else if (sFlag) atomicOr(&P.flags[ch], sFlag);
    }
}

}  // namespace fpcg
