// Device-side building blocks for gfx950 (CDNA4): matrix-core operand traits
// per number format, rounding conversions, wave reductions and the QAM slicer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fpcg {

enum Fmt : int { F64 = 0, F32 = 1, BF16 = 2, F16 = 3, F8 = 4 };

enum : uint32_t { FLAG_NONFINITE = 1u, FLAG_BREAKDOWN = 2u, FLAG_BLOCK_NOT_PD = 4u, FLAG_FP8_SAT = 8u };

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Rounding of an fp32 value to an operand format (round to nearest even).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_bits(float v) {
    __bf16 h = (__bf16)v;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ uint16_t f16_bits(float v) {
    _Float16 h = (_Float16)v;
    return __builtin_bit_cast(uint16_t, h);
}
// two fp32 -> two halves of one word (a in the low half), both rounded to
// nearest even; one packed conversion (v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f16x2_bits(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, f16x2));
}
__device__ __forceinline__ uint32_t bf16x2_bits(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
// two fp32 -> two OCP e4m3 bytes (low 16 bits of the result)
__device__ __forceinline__ uint32_t fp8x2_bits(float a, float b) {
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) {
    return (float)__builtin_bit_cast(_Float16, h);
}
__device__ __forceinline__ float fp8_to_f32(uint32_t byte) {
    return __builtin_amdgcn_cvt_f32_fp8((int)byte, 0);
}

// one element rounded to an operand format, as the bits that format stores
template <int FMT> __device__ __forceinline__ uint32_t op_bits(float v);
template <> __device__ __forceinline__ uint32_t op_bits<F8>(float v) { return fp8x2_bits(v, 0.f) & 0xffu; }
template <> __device__ __forceinline__ uint32_t op_bits<F16>(float v) { return f16_bits(v); }
template <> __device__ __forceinline__ uint32_t op_bits<BF16>(float v) { return bf16_bits(v); }

// fmt(v): the value v rounded to fmt and widened back to fp32
__device__ __forceinline__ float round_to(float v, int fmt) {
    switch (fmt) {
        case BF16: return bf16_to_f32(bf16_bits(v));
        case F16: return f16_to_f32(f16_bits(v));
        case F8: return fp8_to_f32(fp8x2_bits(v, 0.f) & 0xffu);
        default: return v;
    }
}

// Exact power-of-two scale 2^e with 2^e * amax <= 448 < 2^(e+1) * amax
// (fp8 e4m3 range), e clamped to [-126, 126]; amax <= 0 or not finite -> e = 0.
__device__ __forceinline__ int fp8_scale_exp(float amax) {
    if (!(amax > 0.f) || !__builtin_isfinite(amax)) return 0;
    int ea;
    float ma = frexpf(amax, &ea);                 // amax = ma 2^ea, ma in [0.5, 1)
    int e = (ma <= 0.875f) ? (9 - ea) : (8 - ea); // 448 = 0.875 2^9
    return e < -126 ? -126 : (e > 126 ? 126 : e);
}

// ---------------------------------------------------------------------------
// Matrix-core operand traits.  One 16x16 output tile; lane l holds column
// l % 16 and four rows crow(l / 16, i), i = 0..3 (4*g + i for the fp32-
// accumulating shapes, 4*i + g for the f64 shape).  The A and B operands
// of one instruction carry KPL contraction values per lane; both operands use
// the same lane/slot -> k assignment, so any consistent packing of the
// contraction index is valid.
// ---------------------------------------------------------------------------
template <int FMT, int KPL> struct Op;

template <> struct Op<F64, 1> {
    using work = double;
    using frag = double;
    using acc = f64x4;
    // output tile: lane group g, accumulator element i -> row 4*i + g (f64 shape)
    __device__ static __forceinline__ int crow(int g, int i) { return 4 * i + g; }
    __device__ static __forceinline__ void cinv(int m, int& g, int& i) { g = m & 3; i = m >> 2; }
    static constexpr int KPL = 1;
    __device__ static __forceinline__ acc mfma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag pack(const work* v, float) { return v[0]; }
    __device__ static __forceinline__ frag neg(frag a) { return -a; }
};

template <> struct Op<F32, 1> {
    using work = float;
    using frag = float;
    using acc = f32x4;
    // output tile: lane group g, accumulator element i -> row crow(g, i); cinv inverts it
    __device__ static __forceinline__ int crow(int g, int i) { return 4 * g + i; }
    __device__ static __forceinline__ void cinv(int m, int& g, int& i) { g = m >> 2; i = m & 3; }
    static constexpr int KPL = 1;
    __device__ static __forceinline__ acc mfma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag pack(const work* v, float) { return v[0]; }
    __device__ static __forceinline__ frag neg(frag a) { return -a; }
};

template <> struct Op<BF16, 8> {
    using work = float;
    using frag = u32x4;
    using acc = f32x4;
    // output tile: lane group g, accumulator element i -> row crow(g, i); cinv inverts it
    __device__ static __forceinline__ int crow(int g, int i) { return 4 * g + i; }
    __device__ static __forceinline__ void cinv(int m, int& g, int& i) { g = m >> 2; i = m & 3; }
    static constexpr int KPL = 8;
    __device__ static __forceinline__ acc mfma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag pack(const float* v, float s) {
        frag r;
#pragma unroll
        for (int j = 0; j < 4; ++j) r[j] = bf16x2_bits(v[2 * j] * s, v[2 * j + 1] * s);
        return r;
    }
    __device__ static __forceinline__ frag neg(frag a) { return a ^ 0x80008000u; }
};

template <> struct Op<BF16, 4> {
    using work = float;
    using frag = u32x2;
    using acc = f32x4;
    // output tile: lane group g, accumulator element i -> row crow(g, i); cinv inverts it
    __device__ static __forceinline__ int crow(int g, int i) { return 4 * g + i; }
    __device__ static __forceinline__ void cinv(int m, int& g, int& i) { g = m >> 2; i = m & 3; }
    static constexpr int KPL = 4;
    __device__ static __forceinline__ acc mfma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(i16x4, a), __builtin_bit_cast(i16x4, b), c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag pack(const float* v, float s) {
        frag r;
#pragma unroll
        for (int j = 0; j < 2; ++j) r[j] = bf16x2_bits(v[2 * j] * s, v[2 * j + 1] * s);
        return r;
    }
    __device__ static __forceinline__ frag neg(frag a) { return a ^ 0x80008000u; }
};

template <> struct Op<F16, 8> {
    using work = float;
    using frag = u32x4;
    using acc = f32x4;
    // output tile: lane group g, accumulator element i -> row crow(g, i); cinv inverts it
    __device__ static __forceinline__ int crow(int g, int i) { return 4 * g + i; }
    __device__ static __forceinline__ void cinv(int m, int& g, int& i) { g = m >> 2; i = m & 3; }
    static constexpr int KPL = 8;
    __device__ static __forceinline__ acc mfma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag pack(const float* v, float s) {
        frag r;
#pragma unroll
        for (int j = 0; j < 4; ++j) r[j] = f16x2_bits(v[2 * j] * s, v[2 * j + 1] * s);
        return r;
    }
    __device__ static __forceinline__ frag neg(frag a) { return a ^ 0x80008000u; }
};

template <> struct Op<F16, 4> {
    using work = float;
    using frag = u32x2;
    using acc = f32x4;
    // output tile: lane group g, accumulator element i -> row crow(g, i); cinv inverts it
    __device__ static __forceinline__ int crow(int g, int i) { return 4 * g + i; }
    __device__ static __forceinline__ void cinv(int m, int& g, int& i) { g = m >> 2; i = m & 3; }
    static constexpr int KPL = 4;
    __device__ static __forceinline__ acc mfma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(f16x4, a), __builtin_bit_cast(f16x4, b), c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag pack(const float* v, float s) {
        frag r;
#pragma unroll
        for (int j = 0; j < 2; ++j) r[j] = f16x2_bits(v[2 * j] * s, v[2 * j + 1] * s);
        return r;
    }
    __device__ static __forceinline__ frag neg(frag a) { return a ^ 0x80008000u; }
};

template <> struct Op<F8, 8> {
    using work = float;
    using frag = u32x2;
    using acc = f32x4;
    // output tile: lane group g, accumulator element i -> row crow(g, i); cinv inverts it
    __device__ static __forceinline__ int crow(int g, int i) { return 4 * g + i; }
    __device__ static __forceinline__ void cinv(int m, int& g, int& i) { g = m >> 2; i = m & 3; }
    static constexpr int KPL = 8;
    __device__ static __forceinline__ acc mfma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag pack(const float* v, float s) {
        frag r;
#pragma unroll
        for (int j = 0; j < 2; ++j)
            r[j] = fp8x2_bits(v[4 * j] * s, v[4 * j + 1] * s) | (fp8x2_bits(v[4 * j + 2] * s, v[4 * j + 3] * s) << 16);
        return r;
    }
    __device__ static __forceinline__ frag neg(frag a) { return a ^ 0x80808080u; }
};

// ---------------------------------------------------------------------------
// Column reductions over the four 16-lane groups of a wave, on the VALU lane
// swaps of gfx950: v_permlane16_swap exchanges 16-lane rows 0<->1 and 2<->3,
// v_permlane32_swap the two 32-lane halves.  After each swap every lane holds
// its own value and its partner's, so lanes l, l^16, l^32, l^48 end with
// bitwise identical results ((v0 + v1) + (v2 + v3) in every lane).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void swap16(uint32_t v, uint32_t& a, uint32_t& b) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    a = r[0]; b = r[1];
}
__device__ __forceinline__ void swap32(uint32_t v, uint32_t& a, uint32_t& b) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    a = r[0]; b = r[1];
}
// both halves of the exchange for float / double: lo = value of the lower
// row (or half) of the pair, hi = value of the upper one
template <int S> __device__ __forceinline__ void pair_of(float v, float& lo, float& hi) {
    uint32_t a, b;
    if constexpr (S == 16) swap16(__float_as_uint(v), a, b); else swap32(__float_as_uint(v), a, b);
    lo = __uint_as_float(a); hi = __uint_as_float(b);
}
template <int S> __device__ __forceinline__ void pair_of(double v, double& lo, double& hi) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    uint32_t a0, b0, a1, b1;
    if constexpr (S == 16) { swap16((uint32_t)u, a0, b0); swap16((uint32_t)(u >> 32), a1, b1); }
    else { swap32((uint32_t)u, a0, b0); swap32((uint32_t)(u >> 32), a1, b1); }
    lo = __longlong_as_double((long long)(((uint64_t)a1 << 32) | a0));
    hi = __longlong_as_double((long long)(((uint64_t)b1 << 32) | b0));
}
// Value of lane J of each group of four lanes (DPP quad_perm [J, J, J, J],
// a VALU move with no LDS round trip); J must fold to a constant.
template <int J> __device__ __forceinline__ uint32_t quad_bcast_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, J * 0x55, 0xF, 0xF, false);
}
template <int J> __device__ __forceinline__ float quad_bcast(float v) {
    return __uint_as_float(quad_bcast_u32<J>(__float_as_uint(v)));
}
template <int J> __device__ __forceinline__ double quad_bcast(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = quad_bcast_u32<J>((uint32_t)u), hi = quad_bcast_u32<J>((uint32_t)(u >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}
template <typename T> __device__ __forceinline__ T quad_bcast(T v, int j) {
    switch (j) {
        case 0: return quad_bcast<0>(v);
        case 1: return quad_bcast<1>(v);
        case 2: return quad_bcast<2>(v);
        default: return quad_bcast<3>(v);
    }
}
template <typename T> __device__ __forceinline__ T col_sum(T v) {
    T lo, hi;
    pair_of<16>(v, lo, hi);
    v = lo + hi;
    pair_of<32>(v, lo, hi);
    return lo + hi;
}
template <typename T> __device__ __forceinline__ T col_max(T v) {
    T lo, hi;
    pair_of<16>(v, lo, hi);
    v = lo > hi ? lo : hi;
    pair_of<32>(v, lo, hi);
    return lo > hi ? lo : hi;
}
template <typename T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        T o = __shfl_xor(v, s);
        v = v > o ? v : o;
    }
    return v;
}

// ---------------------------------------------------------------------------
// QAM slicer: per axis j = clamp(floor((v nu + m) / 2), 0, m - 1), each
// operation rounded (no contraction), decided in the precision of T.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }

template <typename T> __device__ __forceinline__ int slice_axis(T v, T nu, T mm, int m) {
    T t = add_rn(mul_rn(v, nu), mm);
    T j = floor(t * T(0.5));
    const T jc = fmin(fmax(j, T(0)), T(m - 1));      // index clamped to [0, m-1]
    return __builtin_isfinite(j) ? (int)jc : 0;       // a non-finite estimate maps to index 0
}

template <typename T> __device__ __forceinline__ uint8_t slice_label(T re, T im, T nu, T mm, int m, int bits) {
    int ji = slice_axis(re, nu, mm, m);
    int jq = slice_axis(im, nu, mm, m);
    return (uint8_t)((((ji ^ (ji >> 1))) << bits) | (jq ^ (jq >> 1)));
}

// ---------------------------------------------------------------------------
// Range-checked loads through a buffer resource covering [base, base+bytes):
// a byte offset outside that range reads as zero in hardware, so masked
// loads need no branch and every load of a block can be in flight at once.
// ---------------------------------------------------------------------------
typedef uint32_t u32x2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
constexpr uint32_t OOB = 0x80000000u;   // any offset >= the range reads 0
// Cache policy of a buffer access: non-temporal (streaming) for data touched
// once whose 128-byte lines are consumed whole by one access (H rows of a
// multiple of 128 bytes, the staged x_hat chunks); the default policy where
// neighbouring rows share lines (Y rows of R = 14 complex64 values are 112
// bytes: non-temporal loads of them fetched shared lines twice and measured
// 30 us slower at c2).
constexpr int CP_STREAM = 2;

struct Buf {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ Buf(const void* base, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000)) {}
};

template <typename IOT> struct CxB;
// (vector elements are copied to scalars before a bit cast: a bit cast applied
// directly to an ext-vector element reads the vector's first element)
template <> struct CxB<float> {
    static constexpr uint32_t bytes = 8;
    template <int CP = 0, typename T> __device__ static __forceinline__ void load(const Buf& b, uint32_t off, T& re, T& im) {
        const u32x2v v = __builtin_amdgcn_raw_buffer_load_b64(b.r, off, 0, CP);
        const uint32_t lo = v[0], hi = v[1];
        re = (T)__uint_as_float(lo);
        im = (T)__uint_as_float(hi);
    }
    // store re + i im as complex64 (values outside the range are dropped)
    template <typename T> __device__ static __forceinline__ void store(const Buf& b, uint32_t off, T re, T im) {
        const u32x2v v = {__float_as_uint((float)re), __float_as_uint((float)im)};
        __builtin_amdgcn_raw_buffer_store_b64(v, b.r, off, 0, 0);
    }
};
template <> struct CxB<double> {
    static constexpr uint32_t bytes = 16;
    template <int CP = 0, typename T> __device__ static __forceinline__ void load(const Buf& b, uint32_t off, T& re, T& im) {
        const u32x4v v = __builtin_amdgcn_raw_buffer_load_b128(b.r, off, 0, CP);
        const uint64_t a = ((uint64_t)(uint32_t)v[1] << 32) | (uint32_t)v[0];
        const uint64_t c = ((uint64_t)(uint32_t)v[3] << 32) | (uint32_t)v[2];
        re = (T)__longlong_as_double((long long)a);
        im = (T)__longlong_as_double((long long)c);
    }
    // store re + i im as complex128 (values outside the range are dropped)
    template <typename T> __device__ static __forceinline__ void store(const Buf& b, uint32_t off, T re, T im) {
        const uint64_t a = (uint64_t)__double_as_longlong((double)re), c = (uint64_t)__double_as_longlong((double)im);
        const u32x4v v = {(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)c, (uint32_t)(c >> 32)};
        __builtin_amdgcn_raw_buffer_store_b128(v, b.r, off, 0, 0);
    }
};
// 16 and 8 bytes with cache policy CP (values outside the range are dropped)
template <int CP> __device__ __forceinline__ void store_b128(const Buf& b, uint32_t off, u32x4v v) {
    __builtin_amdgcn_raw_buffer_store_b128(v, b.r, off, 0, CP);
}
template <int CP> __device__ __forceinline__ void store_b64(const Buf& b, uint32_t off, u32x2v v) {
    __builtin_amdgcn_raw_buffer_store_b64(v, b.r, off, 0, CP);
}
// one byte (values outside the range are dropped)
__device__ __forceinline__ void store_u8(const Buf& b, uint32_t off, uint8_t v) {
    __builtin_amdgcn_raw_buffer_store_b8(v, b.r, off, 0, 0);
}

// complex element loads/stores for complex64 (float) or complex128 (double) I/O
template <typename IOT> struct Cx;
template <> struct Cx<float> {
    __device__ static __forceinline__ void load(const void* base, int64_t idx, double& re, double& im) {
        float2 v = reinterpret_cast<const float2*>(base)[idx];
        re = v.x; im = v.y;
    }
    __device__ static __forceinline__ void load(const void* base, int64_t idx, float& re, float& im) {
        float2 v = reinterpret_cast<const float2*>(base)[idx];
        re = v.x; im = v.y;
    }
    template <typename T> __device__ static __forceinline__ void store(void* base, int64_t idx, T re, T im) {
        reinterpret_cast<float2*>(base)[idx] = make_float2((float)re, (float)im);
    }
};
template <> struct Cx<double> {
    __device__ static __forceinline__ void load(const void* base, int64_t idx, double& re, double& im) {
        double2 v = reinterpret_cast<const double2*>(base)[idx];
        re = v.x; im = v.y;
    }
    // narrowing load for fp32-path schedules: round to fp32 first (the operand
    // formats are reached from fp32, as the conversion instructions are)
    __device__ static __forceinline__ void load(const void* base, int64_t idx, float& re, float& im) {
        double2 v = reinterpret_cast<const double2*>(base)[idx];
        re = (float)v.x; im = (float)v.y;
    }
    template <typename T> __device__ static __forceinline__ void store(void* base, int64_t idx, T re, T im) {
        reinterpret_cast<double2*>(base)[idx] = make_double2((double)re, (double)im);
    }
};

}  // namespace fpcg
