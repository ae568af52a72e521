// Device-side building blocks of the NMFA hot path for gfx950 (CDNA4).
//
//   * Philox4x32-10 counter-based generator (Salmon et al., SC'11) and the Box-Muller transform
//     that turn (seed, t, replica, spin) into the Gaussian noise N(0, sigma) added to the
//     normalised mean field (paper Sec. II, the field line of Algorithm 1).
//   * The Boltzmann factor -tanh(Phi / T_t) (Algorithm 1, the s-hat line).
//   * Precision traits mapping each precision of the library onto one MFMA instruction with
//     a 16x16 output tile: FP64 (v_mfma_f64_16x16x4_f64), FP32 (v_mfma_f32_16x16x4_f32) and
//     BF16 (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// MFMA 16x16 fragment layouts used throughout (lane l = 0..63, lane group g = l / 16):
//   A (rows x k):  lane l supplies row (l % 16) and KW consecutive k of its lane group.
//   B (k x cols):  lane l supplies col (l % 16) and the same KW k.
//   D (rows x cols): lane l holds col (l % 16) and four rows: 4g .. 4g+3 for the FP32 and BF16
//                    instructions, but g, g+4, g+8, g+12 for v_mfma_f64_16x16x4_f64 (measured
//                    on gfx950). The FP64 path therefore feeds A-operand row slot a with the
//                    actual row 4 (a % 4) + a / 4, which brings the four rows of each lane back to
//                    4g .. 4g+3 (Traits::a_row).
// Because a dot product does not depend on the order of its k terms, lane group g is given the
// contiguous k range [g*Kq, (g+1)*Kq) (Kq = Kp/4) and MFMA step m uses k = g*Kq + m*KW + j;
// every lane then reads contiguous 16-byte chunks from row-major operands.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmfa {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

enum : int { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2, PREC_FP8J_BF16S = 3, PREC_FP8J_FP8S = 4 };

// ------------------------------------------------------------------------------------------
// Philox4x32-10. Counter (q, r, t, 0), key (seed_lo, seed_hi). Each round multiplies words 0
// and 2 by the two Philox constants, and mixes the high halves with words 1, 3 and the key;
// the key advances by the Weyl increments between rounds.
// ------------------------------------------------------------------------------------------
struct Philox4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    // three-input XOR in one instruction (v_bitop3_b32 with truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Philox4{c0, c1, c2, c3};
}

// ------------------------------------------------------------------------------------------
// Gaussian noise, FP32 fast path. Uniforms u = x * 2^-32 + 2^-33 in (0, 1]; Box-Muller with
// sigma folded into the radius: sigma * z(2p) = rho * cos(2 pi u1), rho = sqrt(-2 sigma^2 ln u0).
// v_log_f32 computes log2, v_sin/v_cos_f32 take their argument in revolutions (x -> sin(2 pi x)).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void sigma_gauss4_f32(const Philox4& w, float neg2ln2_sigma2, float z[4]) {
  const float u0 = fmaf((float)w.x0, 0x1p-32f, 0x1p-33f);
  const float u1 = fmaf((float)w.x1, 0x1p-32f, 0x1p-33f);
  const float u2 = fmaf((float)w.x2, 0x1p-32f, 0x1p-33f);
  const float u3 = fmaf((float)w.x3, 0x1p-32f, 0x1p-33f);
  const float rho0 = __builtin_amdgcn_sqrtf(neg2ln2_sigma2 * __builtin_amdgcn_logf(u0));
  const float rho1 = __builtin_amdgcn_sqrtf(neg2ln2_sigma2 * __builtin_amdgcn_logf(u2));
  z[0] = rho0 * __builtin_amdgcn_cosf(u1);
  z[1] = rho0 * __builtin_amdgcn_sinf(u1);
  z[2] = rho1 * __builtin_amdgcn_cosf(u3);
  z[3] = rho1 * __builtin_amdgcn_sinf(u3);
}

// Gaussian noise, FP64 validation path: u = (x + 1/2) 2^-32 exactly, z = sqrt(-2 ln u0) cos(2 pi u1)
// and sin(2 pi u1) with the device math library; the caller multiplies by sigma.
__device__ __forceinline__ void gauss4_f64(const Philox4& w, double z[4]) {
  const double two_pi = 6.283185307179586476925286766559;
  const double u0 = ((double)w.x0 + 0.5) * 0x1p-32;
  const double u1 = ((double)w.x1 + 0.5) * 0x1p-32;
  const double u2 = ((double)w.x2 + 0.5) * 0x1p-32;
  const double u3 = ((double)w.x3 + 0.5) * 0x1p-32;
  const double rho0 = sqrt(-2.0 * log(u0));
  const double rho1 = sqrt(-2.0 * log(u2));
  double s, c;
  sincos(two_pi * u1, &s, &c);
  z[0] = rho0 * c;
  z[1] = rho0 * s;
  sincos(two_pi * u3, &s, &c);
  z[2] = rho1 * c;
  z[3] = rho1 * s;
}

// -tanh(y) with e = exp(2y) computed as 2^(y * 2 log2 e); the caller passes a = 2 log2(e) * y.
// 2 / (1 + e) - 1 saturates correctly: e -> inf gives -1, e -> 0 gives +1.
__device__ __forceinline__ float neg_tanh_from_exp2_arg(float a) {
  const float e = __builtin_amdgcn_exp2f(a);
  return fmaf(2.0f, __builtin_amdgcn_rcpf(1.0f + e), -1.0f);
}

// ------------------------------------------------------------------------------------------
// Precision traits.
// ------------------------------------------------------------------------------------------
template <int P>
struct Traits;

template <>
struct Traits<PREC_FP64> {
  using op_t = double;    // MFMA operand element
  using acc_t = double;   // accumulator / state element
  using frag_t = double;  // per-lane MFMA operand
  using acc4_t = f64x4;
  static constexpr int KW = 1;  // k values per lane per MFMA
  __device__ static __forceinline__ acc4_t mfma(frag_t a, frag_t b, acc4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // actual row (within a 16-row tile) that A-operand row slot c must carry
  __device__ static __forceinline__ int a_row(int c) { return 4 * (c & 3) + (c >> 2); }
};

template <>
struct Traits<PREC_FP32> {
  using op_t = float;
  using acc_t = float;
  using frag_t = float;
  using acc4_t = f32x4;
  static constexpr int KW = 1;
  __device__ static __forceinline__ acc4_t mfma(frag_t a, frag_t b, acc4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int a_row(int c) { return c; }
};

template <>
struct Traits<PREC_BF16> {
  using op_t = __bf16;
  using acc_t = float;
  using frag_t = bf16x8;
  using acc4_t = f32x4;
  static constexpr int KW = 8;
  __device__ static __forceinline__ acc4_t mfma(frag_t a, frag_t b, acc4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int a_row(int c) { return c; }
};

// FP32 -> BF16 round to nearest even (finite inputs only: states are bounded by 1).
__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }

}  // namespace nmfa

namespace nmfa {

// FP8 E4M3 (OCP "fn" variant: bias 7, no infinities, 0x7f/0xff = NaN) to float, exactly.
__device__ __forceinline__ float fp8e4m3_to_float(uint32_t byte) {
  const uint32_t sign = (byte & 0x80u) << 24;
  const uint32_t e = (byte >> 3) & 0xfu;
  const uint32_t m = byte & 0x7u;
  float mag;
  if (e == 0) {
    mag = (float)m * 0x1p-9f;  // subnormal: m/8 * 2^-6
  } else if (e == 15 && m == 7) {
    mag = __builtin_nanf("");
  } else {
    mag = __uint_as_float(((e + 120u) << 23) | (m << 20));
  }
  return __uint_as_float(__float_as_uint(mag) | sign);
}

}  // namespace nmfa
