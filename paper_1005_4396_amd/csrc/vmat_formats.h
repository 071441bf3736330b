// Storage formats of D on the device and their decode to FP32.
//
// FP32 values are exact; BF16/FP16 are round-to-nearest-even encodings of the
// FP32 value; FP8 is OCP E4M3 (bias 7, 3 mantissa bits, subnormals at exponent
// field 0, max 448, no infinities) of D_ij / s_i with a per-row FP32 scale.
// Every decoded value is exactly representable in FP32, and FP32 x FP32
// products are exact in FP64, so the only approximation of the reduced formats
// is the encoding itself.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vmat {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

enum Fmt { FMT_F32 = 0, FMT_F16 = 1, FMT_BF16 = 2, FMT_FP8 = 3 };

__host__ __device__ inline int fmt_bytes(int fmt) {
    return fmt == FMT_F32 ? 4 : (fmt == FMT_FP8 ? 1 : 2);
}

// ---- decode
__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) {
    return __uint_as_float(bits16 << 16);
}

__device__ __forceinline__ float f16_to_f32(uint32_t bits16) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
}

// E4M3 code -> float.  Normal: (1 + m/8) 2^(e-7); subnormal: m 2^-9.
__device__ __forceinline__ float e4m3_to_f32(uint32_t code) {
    const uint32_t e = (code >> 3) & 0xF, m = code & 0x7, s = (code & 0x80) << 24;
    const float sub = (float)m * 0.001953125f;  // m * 2^-9
    const float nrm = __uint_as_float(((e + 120u) << 23) | (m << 20));
    return __uint_as_float(__float_as_uint(e ? nrm : sub) | s);
}

// ---- encode (used once, when the handle is built)
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t b = __float_as_uint(f);
    uint32_t lsb = (b >> 16) & 1u;
    return (uint16_t)((b + 0x7FFFu + lsb) >> 16);
}

__device__ __forceinline__ uint16_t f32_to_f16_rne(float f) {
    return __builtin_bit_cast(uint16_t, (_Float16)f);  // IEEE round to nearest even
}

// v in [0, 448] -> nearest E4M3 code, ties to the even code.  The decision is
// taken on the FP64 value of v.
__device__ __forceinline__ uint8_t f64_to_e4m3_rne(double v) {
    if (!(v > 0.0)) return 0;
    if (v >= 448.0) return 0x7E;
    // largest code whose value <= v: binary search over the 127 finite codes
    int lo = 0, hi = 126;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((double)e4m3_to_f32((uint32_t)mid) <= v) lo = mid; else hi = mid - 1;
    }
    if (lo == 126) return 126;
    const double a = (double)e4m3_to_f32((uint32_t)lo);
    const double b = (double)e4m3_to_f32((uint32_t)(lo + 1));
    if (a == v) return (uint8_t)lo;
    const double da = v - a, db = b - v;
    if (db < da) return (uint8_t)(lo + 1);
    if (da < db) return (uint8_t)lo;
    return (uint8_t)(((lo + 1) & 1) == 0 ? lo + 1 : lo);
}

// ---- 4-value loads for quad CSR
// load: non-temporal (a stream read once per product); ld: an ordinary load,
// for data that other waves read again soon (kept in the caches).
template <int FMT> struct Quad;

template <> struct Quad<FMT_F32> {
    using raw_t = f32x4;
    __device__ __forceinline__ static raw_t raw(const void* base, int64_t q) {
        return __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(base) + q);
    }
    __device__ __forceinline__ static float4 dec(f32x4 v) { return make_float4(v.x, v.y, v.z, v.w); }
    __device__ __forceinline__ static float4 load(const void* base, int64_t q) {
        return dec(__builtin_nontemporal_load(reinterpret_cast<const f32x4*>(base) + q));
    }
    __device__ __forceinline__ static float4 ld(const void* base, int64_t q) {
        return dec(reinterpret_cast<const f32x4*>(base)[q]);
    }
};

template <> struct Quad<FMT_BF16> {
    using raw_t = u32x2;
    __device__ __forceinline__ static raw_t raw(const void* base, int64_t q) {
        return __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(base) + q);
    }
    __device__ __forceinline__ static float4 dec(u32x2 u) {
        return make_float4(bf16_to_f32(u.x & 0xFFFFu), bf16_to_f32(u.x >> 16),
                           bf16_to_f32(u.y & 0xFFFFu), bf16_to_f32(u.y >> 16));
    }
    __device__ __forceinline__ static float4 load(const void* base, int64_t q) {
        return dec(__builtin_nontemporal_load(reinterpret_cast<const u32x2*>(base) + q));
    }
    __device__ __forceinline__ static float4 ld(const void* base, int64_t q) {
        return dec(reinterpret_cast<const u32x2*>(base)[q]);
    }
};

template <> struct Quad<FMT_F16> {
    using raw_t = u32x2;
    __device__ __forceinline__ static raw_t raw(const void* base, int64_t q) {
        return __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(base) + q);
    }
    __device__ __forceinline__ static float4 dec(u32x2 u) {
        return make_float4(f16_to_f32(u.x & 0xFFFFu), f16_to_f32(u.x >> 16),
                           f16_to_f32(u.y & 0xFFFFu), f16_to_f32(u.y >> 16));
    }
    __device__ __forceinline__ static float4 load(const void* base, int64_t q) {
        return dec(__builtin_nontemporal_load(reinterpret_cast<const u32x2*>(base) + q));
    }
    __device__ __forceinline__ static float4 ld(const void* base, int64_t q) {
        return dec(reinterpret_cast<const u32x2*>(base)[q]);
    }
};

// The hardware conversion (two codes per instruction) gives the same bits as
// e4m3_to_f32 on every finite code; stored codes never exceed 0x7E.
template <> struct Quad<FMT_FP8> {
    using raw_t = uint32_t;
    __device__ __forceinline__ static raw_t raw(const void* base, int64_t q) {
        return __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(base) + q);
    }
    __device__ __forceinline__ static float4 dec(uint32_t u) {
        const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)u, false);
        const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)u, true);
        return make_float4(lo.x, lo.y, hi.x, hi.y);
    }
    __device__ __forceinline__ static float4 load(const void* base, int64_t q) {
        return dec(__builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(base) + q));
    }
    __device__ __forceinline__ static float4 ld(const void* base, int64_t q) {
        return dec(reinterpret_cast<const uint32_t*>(base)[q]);
    }
};

}  // namespace vmat
