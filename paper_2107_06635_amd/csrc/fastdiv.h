// Division by a divisor fixed at launch without the software divide: for
// 1 <= d < 2^31 and 0 <= x < 2^31, x / d = (x * m) >> (32 + s) with
// s = ceil(log2 d) and m = ceil(2^(32+s) / d) (< 2^33).  With e = m d -
// 2^(32+s) < d <= 2^s the product overshoots x / d by x e / (d 2^(32+s)) <
// 1 / (2 d), less than the distance of x / d to the next integer.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define NTU_FD_HD __host__ __device__ __forceinline__
#else
#define NTU_FD_HD static inline
#endif

typedef struct FastDiv {
  uint64_t m;
  uint32_t d;
  uint32_t s;
} FastDiv;

NTU_FD_HD FastDiv make_fastdiv(uint32_t d) {
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  const uint64_t p = 1ull << (32 + s);
  FastDiv f;
  f.m = (p + d - 1) / d;
  f.d = d;
  f.s = s;
  return f;
}
NTU_FD_HD uint32_t fdiv(uint32_t x, FastDiv f) { return (uint32_t)((x * f.m) >> (32 + f.s)); }
NTU_FD_HD uint32_t fmod_(uint32_t x, FastDiv f) { return x - fdiv(x, f) * f.d; }
