// Storage formats of the buckets: IEEE binary16, bfloat16 (the upper half of
// binary32) and OCP FP8 E4M3FN (bias 7, no infinities, largest finite 448).
//
// Encoding rounds a finite FP64 value straight to the format, to nearest with
// ties to even, keeping subnormals (no intermediate binary32 rounding, which
// could round twice).  Decoding is exact into binary32.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bspai {

// Round |x| (a finite double) to a format with P significand bits and minimum
// normal exponent EMIN.  Returns the integer significand r and the exponent
// qexp of its unit, value = r * 2^qexp, with r <= 2^P.
template <int P, int EMIN>
__host__ __device__ inline uint64_t round_significand(double x, int *qexp) {
  uint64_t bits = __builtin_bit_cast(uint64_t, x);
  int ebits = (int)((bits >> 52) & 0x7FF);
  uint64_t frac = bits & ((1ull << 52) - 1);
  if (ebits == 0 && frac == 0) {
    *qexp = EMIN - (P - 1);
    return 0;
  }
  // double subnormals lie far below every target format's range
  int e = ebits ? ebits - 1023 : -1022;
  uint64_t mant = ebits ? (frac | (1ull << 52)) : frac;  // value = mant * 2^(e-52)
  int q = (e < EMIN ? EMIN : e) - (P - 1);                 // exponent of the target's unit
  int shift = q - (e - 52);                                // bits of mant below the unit
  *qexp = q;
  if (shift <= 0) return mant << (-shift);                // not reached for P <= 24
  if (shift > 53) return 0;                                // below half a unit
  uint64_t r = mant >> shift;
  uint64_t rem = mant & ((shift == 64 ? 0 : (1ull << shift)) - 1);
  uint64_t half = 1ull << (shift - 1);
  if (rem > half || (rem == half && (r & 1ull))) r++;
  return r;
}

// Code of a format with P significand bits, EBITS exponent bits and bias BIAS.
template <int P, int EMIN, int EBITS, int BIAS>
__host__ __device__ inline uint32_t encode_rne(double x) {
  uint32_t sign = (uint32_t)(__builtin_bit_cast(uint64_t, x) >> 63);
  int qexp;
  uint64_t r = round_significand<P, EMIN>(x, &qexp);
  uint32_t code;
  if (r < (1ull << (P - 1))) {
    code = (uint32_t)r;  // subnormal (or zero): exponent field 0
  } else {
    int lead = qexp + (P - 1);
    if (r == (1ull << P)) {  // rounded up into the next binade
      r >>= 1;
      lead += 1;
    }
    code = ((uint32_t)(lead + BIAS) << (P - 1)) | (uint32_t)(r - (1ull << (P - 1)));
  }
  return code | (sign << (EBITS + P - 1));
}

__host__ __device__ inline uint16_t encode_f16(double x) { return (uint16_t)encode_rne<11, -14, 5, 15>(x); }
__host__ __device__ inline uint16_t encode_bf16(double x) { return (uint16_t)encode_rne<8, -126, 8, 127>(x); }
__host__ __device__ inline uint8_t encode_e4m3(double x) { return (uint8_t)encode_rne<4, -6, 4, 7>(x); }
__host__ __device__ inline float encode_f32(double x) {
  return __builtin_bit_cast(float, encode_rne<24, -126, 8, 127>(x));
}

__host__ __device__ inline float decode_f16(uint16_t h) {
  uint32_t s = (uint32_t)(h & 0x8000u) << 16;
  uint32_t e = (h >> 10) & 0x1Fu, m = h & 0x3FFu;
  float v;
  if (e == 0)
    v = (float)m * 0x1p-24f;
  else
    v = __builtin_bit_cast(float, ((e + 112u) << 23) | (m << 13));
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) | s);
}

__host__ __device__ inline float decode_bf16(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

__host__ __device__ inline float decode_e4m3(uint8_t c) {
  uint32_t s = (uint32_t)(c & 0x80u) << 24;
  uint32_t e = (c >> 3) & 0xFu, m = c & 7u;
  float v = e ? __builtin_bit_cast(float, ((e + 120u) << 23) | (m << 20)) : (float)m * 0x1p-9f;
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) | s);
}

}  // namespace bspai
