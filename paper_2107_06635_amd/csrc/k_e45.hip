// The two transfer products of the environment contraction (Fig. 4(c,d)),
// fused, in split precision on the gfx950 matrix cores (complex case):
//   L1[a a'][j][b b'] = sum_{t t'} Left[a a'][b b'][t t'] EtopT[j][t t']
//   L2[a a'][j][k]    = sum_{b b'} L1[a a'][j][b b'] EbotT[k][b b']
// For fixed (item, a, a') both are products of n x n complex matrices,
// n = D^2.  One workgroup per (item, a, a') holds the Left block in shared
// memory as bfloat16 pieces, multiplies it by EtopT, keeps the L1 block in
// shared memory (as the A operand of the second product) and writes the L2
// block over the Left block it came from; L1 never reaches HBM.
// EtopT and EbotT are the B operands of every workgroup of an item: they are
// real-embedded, split and stored once per item in the register order of
// the MFMA B fragments (one 16-byte load per lane and fragment), and stay in
// the L2 cache of the XCD that runs the item's workgroups.
// Real embedding as in the tiled products: an A row interleaves (re, im)
// along K; complex row j of B gives real rows 2j = (re, -im) and
// 2j + 1 = (im, re); outputs interleave (re, im).
// n is padded to NPAD (a multiple of 16): the padded rows and columns of
// both operands are zero, so the padded parts of every product are zero.
#include "kernels.h"
#include "mfma_gemm.h"
#include "split_mfma.h"

namespace ntu {

// Fragment counts of one n x n complex B operand padded to NPAD:
// NPAD / 8 real column tiles of 16, NPAD / 16 steps of 32 real K.
NTU_HD int e45_frag_elems(int npad, int nplanes) { return (npad / 8) * (npad / 16) * nplanes * 512; }

NTU_HD int e45_npad(int D) { return ((D * D + 15) / 16) * 16; }

// frag[item][m][tile][step][piece][lane][8]  (m = 0: EtopT, 1: EbotT)
// value (lane, e) of fragment (tile, step): real B row 16 tile + lane % 16,
// real k 32 step + 8 (lane / 16) + e
template <int PREC>
__global__ void __launch_bounds__(256) k_e45_prep(int n, int npad, const cd* __restrict__ ETT,
                                                  const cd* __restrict__ EBT, long long es,
                                                  typename SplitTraits<PREC>::E* __restrict__ frag) {
  using E = typename SplitTraits<PREC>::E;
  constexpr int NP = SplitTraits<PREC>::NT;
  const int item = blockIdx.y, m = blockIdx.z;
  const cd* Em = (m == 0 ? ETT : EBT) + (size_t)item * es;
  const int KS = npad / 16;
  const int per_m = e45_frag_elems(npad, NP);
  E* out = frag + ((size_t)item * 2 + m) * per_m;
  const int nval = per_m / NP;  // values per piece
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nval; v += gridDim.x * blockDim.x) {
    const int e = v & 7, lane = (v >> 3) & 63, f = v >> 9;
    const int tile = f / KS, step = f % KS;
    const int nr = 16 * tile + (lane & 15), kr = 32 * step + 8 * (lane >> 4) + e;
    const int j = nr >> 1, kc = kr >> 1;
    float x = 0.0f;
    if (j < n && kc < n) {
      const cd z = Em[(size_t)j * n + kc];
      const float re = (float)z.x, im = (float)z.y;
      x = (nr & 1) == 0 ? ((kr & 1) == 0 ? re : -im) : ((kr & 1) == 0 ? im : re);
    }
    E t[NP];
    split_value<PREC>(x, t);
#pragma unroll
    for (int p = 0; p < NP; ++p) out[((size_t)(f * NP + p) * 64 + lane) * 8 + e] = t[p];
  }
}

struct alignas(4) bf16pair { __bf16 v[2]; };

// NPAD / 16 waves; wave w computes real output columns [32 w, 32 w + 32) of
// both products, all NPAD rows.  Workgroups are dealt to the 8 XCDs
// round-robin by id; the order puts an item's workgroups on one XCD.
// H: the Left blocks (FP32 (re, im) pairs), item stride hs complex elements,
// (a a') block at (a R + a') n^2; overwritten by the L2 blocks.
template <int PREC, int NPAD>
__global__ void __launch_bounds__(NPAD * 4) k_e45(int n, int R2, int nwork, float* H, long long hs,
                                                  const __bf16* __restrict__ frag) {
  constexpr int NP = SplitTraits<PREC>::NT;
  constexpr int NACC = (PREC == NTU_PREC_BF16X6) ? 3 : 2;
  constexpr int MT = NPAD / 16, KS = NPAD / 16;
  constexpr int LD = 2 * NPAD + 8;
  __shared__ __attribute__((aligned(16))) __bf16 sA[NP][NPAD][LD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int per = (nwork + 7) / 8;
  const int q = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (q >= nwork) return;
  const int item = q / R2, pair = q % R2;
  float* X = H + ((size_t)item * hs + (size_t)pair * n * n) * 2;
  const int per_m = e45_frag_elems(NPAD, NP);
  const __bf16* F1 = frag + (size_t)item * 2 * per_m;
  const __bf16* F2 = F1 + per_m;

  // Left block -> pieces in shared memory (zero padded)
  for (int e = tid; e < NPAD * NPAD; e += blockDim.x) {
    const int r = e / NPAD, c = e % NPAD;
    float re = 0.0f, im = 0.0f;
    if (r < n && c < n) {
      const float2 z = *(const float2*)&X[2 * ((size_t)r * n + c)];
      re = z.x; im = z.y;
    }
    __bf16 tr[NP], ti[NP];
    split_value<PREC>(re, tr);
    split_value<PREC>(im, ti);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      bf16pair v;
      v.v[0] = tr[p]; v.v[1] = ti[p];
      *(bf16pair*)&sA[p][r][2 * c] = v;
    }
  }
  __syncthreads();

  f32x4 acc[NACC][MT][2];
  auto product = [&](const __bf16* F) {
#pragma unroll
    for (int c = 0; c < NACC; ++c)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[c][mt][y] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      bf16x8 b[2][NP];
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int p = 0; p < NP; ++p)
          b[y][p] = *(const bf16x8*)(F + ((size_t)(((2 * w + y) * KS + ks) * NP + p) * 64 + lane) * 8);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        bf16x8 a[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) a[p] = *(const bf16x8*)&sA[p][16 * mt + (lane & 15)][32 * ks + 8 * (lane >> 4)];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          acc[0][mt][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[y][0], acc[0][mt][y], 0, 0, 0);
          acc[1][mt][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[y][1], acc[1][mt][y], 0, 0, 0);
          acc[1][mt][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[y][0], acc[1][mt][y], 0, 0, 0);
          if constexpr (NACC == 3) {
            acc[2][mt][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[y][2], acc[2][mt][y], 0, 0, 0);
            acc[2][mt][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[y][1], acc[2][mt][y], 0, 0, 0);
            acc[2][mt][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[y][0], acc[2][mt][y], 0, 0, 0);
          }
        }
      }
    }
  };
  auto value = [&](int mt, int y, int v) -> float {
    double s = (double)acc[0][mt][y][v];
    if constexpr (NACC == 3) s += (double)acc[1][mt][y][v] + (double)acc[2][mt][y][v];
    else s += (double)acc[1][mt][y][v];
    return (float)s;
  };

  product(F1);
  __syncthreads();  // every wave has read the Left pieces
  // L1 block -> shared memory as the A operand of the second product:
  // output (row b b', real column 2 j + c) -> A row j, real k 2 (b b') + c
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int bb = 16 * mt + 4 * (lane >> 4) + v;
        const int jr = 32 * w + 16 * y + (lane & 15);
        __bf16 t[NP];
        split_value<PREC>(value(mt, y, v), t);
#pragma unroll
        for (int p = 0; p < NP; ++p) sA[p][jr >> 1][2 * bb + (jr & 1)] = t[p];
      }
  __syncthreads();
  product(F2);
  // L2 block over the Left block: row j, real column kr
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 16 * mt + 4 * (lane >> 4) + v;
        const int kr = 32 * w + 16 * y + (lane & 15);
        if (j < n && kr < 2 * n) X[(size_t)j * 2 * n + kr] = value(mt, y, v);
      }
}

bool e45_supported(bool cplx, int precision, int D) {
  return cplx && (precision == NTU_PREC_BF16X3 || precision == NTU_PREC_BF16X6) && D * D <= 64;
}

size_t e45_frag_bytes(int precision, int batch, int D) {
  const int np = precision == NTU_PREC_BF16X6 ? 3 : 2;
  return (size_t)batch * 2 * e45_frag_elems(e45_npad(D), np) * sizeof(__bf16);
}

template <int PREC>
static hipError_t e45_run(int batch, int D, int R, const void* ETT, const void* EBT, long long es, void* H,
                          long long hs, void* frag, hipStream_t st) {
  const int n = D * D, npad = e45_npad(D);
  constexpr int NP = SplitTraits<PREC>::NT;
  const int nval = e45_frag_elems(npad, NP) / NP;
  dim3 gp((nval + 255) / 256, batch, 2);
  hipLaunchKernelGGL(k_e45_prep<PREC>, gp, dim3(256), 0, st, n, npad, (const cd*)ETT, (const cd*)EBT, es,
                     (__bf16*)frag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nwork = batch * R * R;
  dim3 g(8 * ((nwork + 7) / 8));  // the XCD order maps [0, 8 ceil(nwork / 8)) onto the work
  switch (npad) {
    case 16: hipLaunchKernelGGL((k_e45<PREC, 16>), g, dim3(64), 0, st, n, R * R, nwork, (float*)H, hs, (const __bf16*)frag); break;
    case 32: hipLaunchKernelGGL((k_e45<PREC, 32>), g, dim3(128), 0, st, n, R * R, nwork, (float*)H, hs, (const __bf16*)frag); break;
    case 48: hipLaunchKernelGGL((k_e45<PREC, 48>), g, dim3(192), 0, st, n, R * R, nwork, (float*)H, hs, (const __bf16*)frag); break;
    case 64: hipLaunchKernelGGL((k_e45<PREC, 64>), g, dim3(256), 0, st, n, R * R, nwork, (float*)H, hs, (const __bf16*)frag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_e45(int precision, int batch, int D, int R, const void* ETT, const void* EBT, long long es, void* H,
                      long long hs, void* frag, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (D * D > 64) return hipErrorInvalidValue;
  if (precision == NTU_PREC_BF16X6) return e45_run<NTU_PREC_BF16X6>(batch, D, R, ETT, EBT, es, H, hs, frag, st);
  if (precision == NTU_PREC_BF16X3) return e45_run<NTU_PREC_BF16X3>(batch, D, R, ETT, EBT, es, H, hs, frag, st);
  return hipErrorNotSupported;
}

}  // namespace ntu
