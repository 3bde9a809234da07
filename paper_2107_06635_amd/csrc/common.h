// Device helpers shared by the libntu kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#define NTU_DEV __device__ __forceinline__
#define NTU_HD __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------
// scalar types: double (real path) and cd (complex, interleaved re/im)
// ---------------------------------------------------------------------------
struct cd {
  double x, y;
};

NTU_HD cd make_cd(double a, double b) { return cd{a, b}; }
NTU_HD cd operator+(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
NTU_HD cd operator-(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
NTU_HD cd operator-(cd a) { return cd{-a.x, -a.y}; }
NTU_HD cd operator*(cd a, cd b) { return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
NTU_HD cd operator*(double s, cd a) { return cd{s * a.x, s * a.y}; }
NTU_HD cd operator*(cd a, double s) { return cd{s * a.x, s * a.y}; }
NTU_HD cd& operator+=(cd& a, cd b) { a.x += b.x; a.y += b.y; return a; }
NTU_HD cd& operator-=(cd& a, cd b) { a.x -= b.x; a.y -= b.y; return a; }

NTU_HD double conjv(double a) { return a; }
NTU_HD cd conjv(cd a) { return cd{a.x, -a.y}; }
NTU_HD double rev(double a) { return a; }
NTU_HD double rev(cd a) { return a.x; }
NTU_HD double imv(double) { return 0.0; }
NTU_HD double imv(cd a) { return a.y; }
NTU_HD double abs2(double a) { return a * a; }
NTU_HD double abs2(cd a) { return a.x * a.x + a.y * a.y; }
NTU_HD double absv(double a) { return fabs(a); }
NTU_HD double absv(cd a) { return hypot(a.x, a.y); }
// conj(a) * b
NTU_HD double cmul(double a, double b) { return a * b; }
NTU_HD cd cmul(cd a, cd b) { return cd{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }
// a * conj(b)
NTU_HD double mulc(double a, double b) { return a * b; }
NTU_HD cd mulc(cd a, cd b) { return cd{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }

template <class T> NTU_HD T zerov();
template <> NTU_HD double zerov<double>() { return 0.0; }
template <> NTU_HD cd zerov<cd>() { return cd{0.0, 0.0}; }
template <class T> NTU_HD T realv(double a);
template <> NTU_HD double realv<double>(double a) { return a; }
template <> NTU_HD cd realv<cd>(double a) { return cd{a, 0.0}; }
// a / |a| (1 for a == 0)
NTU_HD double phasev(double a) { return a < 0 ? -1.0 : 1.0; }
NTU_HD cd phasev(cd a) {
  double m = hypot(a.x, a.y);
  return m > 0 ? cd{a.x / m, a.y / m} : cd{1.0, 0.0};
}
NTU_HD bool finitev(double a) { return isfinite(a); }
NTU_HD bool finitev(cd a) { return isfinite(a.x) && isfinite(a.y); }

template <class T> struct is_cplx { static constexpr bool value = false; };
template <> struct is_cplx<cd> { static constexpr bool value = true; };

// four doubles: the accumulator of a 16 x 16 x 4 FP64 matrix-core product
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// wave / block reductions (wave64)
// ---------------------------------------------------------------------------
// Cross-lane move of a double inside rows of 16 lanes (DPP).  CTRL 0xB1 and
// 0x4E exchange lanes at distance 1 and 2 inside each quad (quad_perm
// [1,0,3,2], [2,3,0,1]), 0x141 mirrors each half-row, 0x140 each row.
template <int CTRL> NTU_DEV double dpp_move(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  int lo = (int)(unsigned)(u & 0xffffffffull), hi = (int)(unsigned)(u >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Sum over each row of 16 lanes, as a butterfly: after each step the lanes of
// the merged group hold bit-identical values, so all 16 lanes agree.
NTU_DEV double row_sum16(double v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  return v;
}
// Value of lane `src` (uniform across the wave, through a scalar register).
NTU_DEV double lane_value(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), src);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Sum over the wave, (r0 + r16) + (r32 + r48) of the row sums read from
// lanes 0, 16, 32, 48 (no LDS permutes); every lane gets the same value.
NTU_DEV double wave_sum(double v) {
  v = row_sum16(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}
// Sum over lanes 0..31 only (rows of a small matrix held one per lane); the
// result is the same scalar on every lane.  Lanes 32..63 do not contribute.
NTU_DEV double lanes32_sum(double v) {
  const double r = row_sum16(v);
  return lane_value(r, 0) + lane_value(r, 16);
}
NTU_DEV cd lanes32_sum(cd v) { return cd{lanes32_sum(v.x), lanes32_sum(v.y)}; }
NTU_DEV double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
NTU_DEV cd wave_sum(cd v) { return cd{wave_sum(v.x), wave_sum(v.y)}; }

// Sum of v over the block; every thread gets the result.  red: >= 64 doubles
// of shared memory.  Contains two barriers.
NTU_DEV double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}
// Largest v over the workgroup (float, wave64, at most 16 waves); red: 16
// floats of shared memory.  Every thread gets the result.
NTU_DEV float wg_maxf(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  float m = red[0];
  for (int i = 1; i < nw; ++i) m = fmaxf(m, red[i]);
  return m;
}

NTU_DEV double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = -INFINITY;
  for (int i = 0; i < nw; ++i) s = fmax(s, red[i]);
  return s;
}

// Sums n values per thread (vals, in registers) over the block into out[0..n)
// (shared memory, visible to all threads on return).  red: >= 16*64 doubles.
// n <= 64.  Uses doubles; complex callers pass re/im interleaved.
NTU_DEV void block_sum_vec(const double* vals, int n, double* red, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  for (int i = 0; i < n; ++i) {
    double v = wave_sum(vals[i]);
    if (lane == 0) red[w * 64 + i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[k * 64 + i];
    out[i] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// three-level index maps: i -> (i0, i1, i2) with i2 fastest
// ---------------------------------------------------------------------------
struct Idx3 {
  int n1, n2;            // sizes of the two inner levels
  long long s0, s1, s2;  // element strides of the three levels
};
NTU_HD Idx3 idx1(long long s) { return Idx3{1, 1, s, 0, 0}; }
NTU_HD Idx3 idx2(int n_in, long long s_out, long long s_in) { return Idx3{1, n_in, s_out, 0, s_in}; }
NTU_HD Idx3 idx3(int n1, int n2, long long s0, long long s1, long long s2) {
  return Idx3{n1, n2, s0, s1, s2};
}
// Offset of index i (0 <= i < 2^32: rows, columns, contraction indices and
// items are all far below that) under the three-level map.  32-bit unsigned
// division; the one-level case needs none.
NTU_HD long long idx_off(const Idx3& x, long long i) {
  if (x.n1 == 1 && x.n2 == 1) return i * x.s0;
  const unsigned u = (unsigned)i, n2 = (unsigned)x.n2, n1 = (unsigned)x.n1;
  const unsigned i2 = u % n2, t = u / n2;
  const unsigned i1 = t % n1, i0 = t / n1;
  return (long long)i0 * x.s0 + (long long)i1 * x.s1 + (long long)i2 * x.s2;
}
