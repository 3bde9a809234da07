// Operand splitting for the split-precision products on the gfx950 matrix
// cores: a value x becomes NT bfloat16 (or float16) pieces whose sum is x to
// about 8 NT bits, and one 16 x 16 x 32 MFMA multiplies 16 x 32 by 32 x 16
// pieces with FP32 accumulation.
#pragma once
#include "common.h"
#include "ntu.h"

namespace ntu {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int PREC> struct SplitTraits;
template <> struct SplitTraits<NTU_PREC_BF16X3> { static constexpr int NT = 2; using E = __bf16; };
template <> struct SplitTraits<NTU_PREC_BF16X6> { static constexpr int NT = 3; using E = __bf16; };
template <> struct SplitTraits<NTU_PREC_FP16X3> { static constexpr int NT = 2; using E = _Float16; };

// split x (already scaled for FP16) into NT pieces
template <int PREC>
NTU_DEV void split_value(float x, typename SplitTraits<PREC>::E* out) {
  using E = typename SplitTraits<PREC>::E;
  if constexpr (PREC == NTU_PREC_FP16X3) {
    E hi = (E)x;
    float r = (x - (float)hi) * 2048.0f;
    out[0] = hi;
    out[1] = (E)r;
  } else if constexpr (PREC == NTU_PREC_BF16X3) {
    E hi = (E)x;
    out[0] = hi;
    out[1] = (E)(x - (float)hi);
  } else {
    E hi = (E)x;
    float r = x - (float)hi;
    E mid = (E)r;
    out[0] = hi;
    out[1] = mid;
    out[2] = (E)(r - (float)mid);
  }
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Split of two values at once (BF16 precisions): piece p of (x0, x1) as one
// packed word (x0 in the low half).  One packed conversion per piece; the
// FP32 value of a piece is its bits shifted or masked into place.
template <int PREC>
NTU_DEV void split_pair(float x0, float x1, unsigned* out) {
  static_assert(PREC == NTU_PREC_BF16X3 || PREC == NTU_PREC_BF16X6, "bfloat16 pieces only");
  constexpr int NT = SplitTraits<PREC>::NT;
#pragma unroll
  for (int p = 0; p < NT; ++p) {
    const unsigned w = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){x0, x1}, bf16x2));
    out[p] = w;
    if (p + 1 < NT) {
      x0 -= __builtin_bit_cast(float, w << 16);
      x1 -= __builtin_bit_cast(float, w & 0xffff0000u);
    }
  }
}

template <int PREC>
NTU_DEV f32x4 mfma(const typename SplitTraits<PREC>::E* a, const typename SplitTraits<PREC>::E* b, f32x4 c) {
  if constexpr (PREC == NTU_PREC_FP16X3) {
    f16x8 va = *(const f16x8*)a, vb = *(const f16x8*)b;
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(va, vb, c, 0, 0, 0);
  } else {
    bf16x8 va = *(const bf16x8*)a, vb = *(const bf16x8*)b;
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, c, 0, 0, 0);
  }
}

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// FP16X3 pieces of two values already scaled into float16's range:
// hi = fp16(x), lo = fp16((x - hi) 2^11) (the residual is exact in FP32, the
// scaling by 2^11 keeps lo in the normal range); one packed word per piece,
// x0 in the low half.  x = hi + 2^-11 lo to about 2^-22 |x|.
NTU_DEV void split_pair_f16(float x0, float x1, unsigned* out) {
  const f16x2 h = __builtin_convertvector((f32x2){x0, x1}, f16x2);
  const float r0 = (x0 - (float)h.x) * 2048.0f, r1 = (x1 - (float)h.y) * 2048.0f;
  const f16x2 l = __builtin_convertvector((f32x2){r0, r1}, f16x2);
  out[0] = __builtin_bit_cast(unsigned, h);
  out[1] = __builtin_bit_cast(unsigned, l);
}

// Power-of-two scale that brings a block whose largest magnitude is m into
// [2^12, 2^13) (float16 holds up to 65504 and is normal from 2^-14 on); 1
// for an empty or zero block.
NTU_DEV float f16_scale(float m) {
  if (!(m > 0.0f) || !isfinite(m)) return 1.0f;
  return ldexpf(1.0f, 12 - ilogbf(m));
}

}  // namespace ntu
