// BF16 / FP16 helpers and MFMA operand vector types for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Conversions round to nearest even, double -> float -> 16 bits, in hardware
// (v_cvt_f32_f64, then v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32 / v_cvt_f16_f32).  The FP32 step
// is kept explicit: the compiler would otherwise fuse the two roundings into one correctly
// rounded f64 -> 16-bit conversion, a long integer sequence.
__device__ __forceinline__ float keep_f32(double v) { return __builtin_canonicalizef((float)v); }

__device__ __forceinline__ uint16_t bf16_bits_f(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint16_t bf16_bits(double v) { return bf16_bits_f(keep_f32(v)); }
__device__ __forceinline__ float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f16_bits_f(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }
__device__ __forceinline__ uint16_t f16_bits(double v) { return f16_bits_f(keep_f32(v)); }
__device__ __forceinline__ float f16_value(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }

// Two values at once (one packed conversion): element a in the low half.
template <bool HALF>
__device__ __forceinline__ uint32_t pack16(double a, double b) {
    const f32x2 v = {keep_f32(a), keep_f32(b)};
    if constexpr (HALF)
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
    else
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
template <bool HALF>
__device__ __forceinline__ double value16(uint32_t bits16) {
    return HALF ? (double)f16_value((uint16_t)bits16) : (double)bf16_value((uint16_t)bits16);
}

}  // namespace wk
