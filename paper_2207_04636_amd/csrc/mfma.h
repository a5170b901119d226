// Matrix-core (MFMA) helpers for gfx950 and their lane layouts.
//
// Lane layouts (wave64), checked on the device with one-hot operands:
//  v_mfma_f64_16x16x4_f64   D[16x16] += A[16x4] B[4x16]
//     A operand: lane l holds A[l % 16][l / 16]
//     B operand: lane l holds B[l / 16][l % 16]
//     D (4 regs): lane l, reg r holds D[4*r + l/16][l % 16]
//  v_mfma_f32_16x16x4_f32   same A/B layout;
//     D (4 regs): lane l, reg r holds D[4*(l/16) + r][l % 16]
//  v_mfma_f32_16x16x32_bf16 A: lane l holds A[l % 16][8*(l/16) + e], e = 0..7
//                            B: lane l holds B[8*(l/16) + e][l % 16]
//     D as for f32.
#pragma once
#include <hip/hip_runtime.h>

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ d4_t mfma_f64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_f32(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_bf16(bf8_t a, bf8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Row of the f64 D fragment held by (lane, reg).
__device__ __forceinline__ int d64_row(int lane, int r) { return 4 * r + (lane >> 4); }
// Row of the f32 D fragment held by (lane, reg).
__device__ __forceinline__ int d32_row(int lane, int r) { return 4 * (lane >> 4) + r; }

__device__ __forceinline__ d4_t zero_d4() { return d4_t{0.0, 0.0, 0.0, 0.0}; }
__device__ __forceinline__ f4_t zero_f4() { return f4_t{0.f, 0.f, 0.f, 0.f}; }

// Wave-wide sum of a double (deterministic butterfly).
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
