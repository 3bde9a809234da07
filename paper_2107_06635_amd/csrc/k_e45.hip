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
#include <type_traits>
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
                                                  typename SplitTraits<PREC>::E* __restrict__ frag,
                                                  const float* __restrict__ escale) {
  using E = typename SplitTraits<PREC>::E;
  constexpr int NP = SplitTraits<PREC>::NT;
  const int item = blockIdx.y, m = blockIdx.z;
  const cd* Em = (m == 0 ? ETT : EBT) + (size_t)item * es;
  // FP16X3: the item's power-of-two scale of this operand (k_e45_scale)
  const float sc = PREC == NTU_PREC_FP16X3 ? escale[item * 2 + m] : 1.0f;
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
    split_value<PREC>(x * sc, t);
#pragma unroll
    for (int p = 0; p < NP; ++p) out[((size_t)(f * NP + p) * 64 + lane) * 8 + e] = t[p];
  }
}

// FP16X3: per item and operand (EtopT, EbotT) the power-of-two scale that
// brings its largest |re|, |im| into [2^12, 2^13).  Grid (batch, 2).
__global__ void __launch_bounds__(256) k_e45_scale(int n, const cd* __restrict__ ETT, const cd* __restrict__ EBT,
                                                   long long es, float* __restrict__ escale) {
  __shared__ float red[16];
  const int item = blockIdx.x, m = blockIdx.y;
  const cd* Em = (m == 0 ? ETT : EBT) + (size_t)item * es;
  float v = 0.0f;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const cd z = Em[e];
    v = fmaxf(v, fmaxf(fabsf((float)z.x), fabsf((float)z.y)));
  }
  v = wg_maxf(v, red);
  if (threadIdx.x == 0) escale[item * 2 + m] = f16_scale(v);
}

// Per-wave pieces shared by the kernels below.  A product's output tile
// of NPAD rows x 2 NPAD real columns is split over NPAD / 16 waves: wave w
// owns real columns [32 w, 32 w + 32) (two 16-wide MFMA tiles, y = 0, 1) of
// every row tile mt.  acc[0][mt][y] accumulates the hi x hi piece products,
// acc[1][mt][y] all smaller ones (their sum is at most 2^-7 of the first, so
// its FP32 rounding is far below that of the result).  The MFMA runs
// with the operands exchanged (it computes the transposed tile), so that
// lane l holds row 16 mt + l % 16 and the four consecutive real columns
// 32 w + 16 y + 4 (l / 16) + v: two whole complex outputs.
// FP16X3: the power-of-two scale of each isometry block (n x K complex
// entries: QXe[a], QXp[a], QYe[b], QYp[b] for a, b < R), once per item, for
// the fused kernels (each block enters R of their workgroups).  The largest
// |re|, |im| of a block, as the workgroups would find it themselves.
__global__ void __launch_bounds__(256) k_e45_blockscale(int n, int K, int R, const cd* __restrict__ QXe,
                                                        const cd* __restrict__ QXp, const cd* __restrict__ QYe,
                                                        const cd* __restrict__ QYp, long long qs,
                                                        float* __restrict__ blk) {
  __shared__ float red[16];
  const int a = blockIdx.x, which = blockIdx.y, item = blockIdx.z;
  const cd* base = which == 0 ? QXe : which == 1 ? QXp : which == 2 ? QYe : QYp;
  const cd* Q = base + (size_t)item * qs + (size_t)a * n * K;
  float v = 0.0f;
  for (int e = threadIdx.x; e < n * K; e += blockDim.x) {
    const cd z = Q[e];
    v = fmaxf(v, fmaxf(fabsf((float)z.x), fabsf((float)z.y)));
  }
  v = wg_maxf(v, red);
  if (threadIdx.x == 0) blk[((size_t)item * 4 + which) * R + a] = f16_scale(v);
}

template <int PREC, int NPAD> struct E45 {
  static constexpr int NP = SplitTraits<PREC>::NT;
  static constexpr bool F16 = PREC == NTU_PREC_FP16X3;
  static constexpr int NACC = 2;
  static constexpr int MT = NPAD / 16, KS = NPAD / 16;
  static constexpr int LD = 2 * NPAD + 8;
  using E = typename SplitTraits<PREC>::E;
  using V8 = typename std::conditional<F16, f16x8, bf16x8>::type;
  using Acc = f32x4[NACC][MT][2];

  static NTU_DEV f32x4 mf(const V8& a, const V8& b, const f32x4& c) {
    if constexpr (F16) return __builtin_amdgcn_mfma_f32_16x16x32_f16(b, a, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a, c, 0, 0, 0);
  }

  // the piece products kept: BF16x3 (hi, lo): hi hi | lo hi + hi lo;
  // BF16x6 (hi, mid, lo): hi hi | lo hi + mid mid + hi lo + mid hi + hi mid
  // (smallest first); FP16x3 (hi, 2^11 lo): hi hi | lo hi + hi lo, the second
  // accumulator weighted by 2^-11 (comb).  FIRST: the accumulators start from zero.
  template <bool FIRST>
  static NTU_DEV void mma(Acc& acc, int mt, int y, const V8 (&a)[NP], const V8 (&b)[NP]) {
    constexpr f32x4 z = {0, 0, 0, 0};
    acc[0][mt][y] = mf(a[0], b[0], FIRST ? z : acc[0][mt][y]);
    f32x4 t = FIRST ? z : acc[1][mt][y];
    if constexpr (NP == 3) {
      t = mf(a[2], b[0], t);
      t = mf(a[1], b[1], t);
      t = mf(a[0], b[2], t);
    }
    t = mf(a[1], b[0], t);
    acc[1][mt][y] = mf(a[0], b[1], t);
  }

  // value v of the output tile (mt, y): the accumulators combined in FP32
  static NTU_DEV float comb(const Acc& acc, int mt, int y, int v) {
    if constexpr (F16) return acc[0][mt][y][v] + acc[1][mt][y][v] * (1.0f / 2048.0f);
    else return acc[0][mt][y][v] + acc[1][mt][y][v];
  }

  static NTU_DEV void split8(const float (&x)[8], V8 (&f)[NP]) {
    unsigned w[NP][4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      unsigned t[NP];
      if constexpr (F16) split_pair_f16(x[2 * h], x[2 * h + 1], t);
      else split_pair<PREC>(x[2 * h], x[2 * h + 1], t);
#pragma unroll
      for (int p = 0; p < NP; ++p) w[p][h] = t[p];
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
      f[p] = __builtin_bit_cast(V8, (u32x4){w[p][0], w[p][1], w[p][2], w[p][3]});
    }
  }

  // FP16X3: scale of the product held in acc (its largest combined entry)
  static NTU_DEV float acc_scale(const Acc& acc, float* red) {
    float v = 0.0f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q) v = fmaxf(v, fabsf(comb(acc, mt, y, q)));
    return f16_scale(wg_maxf(v, red));
  }

  // P[u][u'] = sum_s Qe[u][s] conj(Qp[u'][s]), u, u' < n, s < K (rows of
  // length K, complex), with the operands multiplied by se, sp (FP16X3
  // scales; 1 otherwise).  A fragment: row u = 16 mt + lane % 16, complex
  // s = 16 kq + 4 (lane / 16) + h; B fragment: real row 32 w + 16 y +
  // lane % 16 of the embedding of conj(Qp).
  static NTU_DEV void pair_product(Acc& acc, const cd* __restrict__ Qe, const cd* __restrict__ Qp, int n, int K,
                                   int w, int lane, float se = 1.0f, float sp = 1.0f) {
    const int KQ = (K + 15) / 16;
    for (int kq = 0; kq < KQ; ++kq) {
      const int s0 = 16 * kq + 4 * (lane >> 4);
      V8 b[2][NP];
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int ur = 32 * w + 16 * y + (lane & 15), u = ur >> 1;
        float x[8];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const bool ok = u < n && s0 + h < K;
          const cd z = Qp[ok ? (size_t)u * K + s0 + h : 0];
          float re = ok ? (float)z.x : 0.0f, im = ok ? -(float)z.y : 0.0f;
          if constexpr (F16) {
            re *= sp;
            im *= sp;
          }
          // real row 2u: (re, -im); 2u + 1: (im, re)
          x[2 * h] = (ur & 1) ? im : re;
          x[2 * h + 1] = (ur & 1) ? re : -im;
        }
        split8(x, b[y]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int u = 16 * mt + (lane & 15);
        float x[8];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const bool ok = u < n && s0 + h < K;
          const cd z = Qe[ok ? (size_t)u * K + s0 + h : 0];
          x[2 * h] = ok ? (float)z.x : 0.0f;
          x[2 * h + 1] = ok ? (float)z.y : 0.0f;
          if constexpr (F16) {
            x[2 * h] *= se;
            x[2 * h + 1] *= se;
          }
        }
        V8 a[NP];
        split8(x, a);
        if (kq == 0) {
#pragma unroll
          for (int y = 0; y < 2; ++y) mma<true>(acc, mt, y, a, b[y]);
        } else {
#pragma unroll
          for (int y = 0; y < 2; ++y) mma<false>(acc, mt, y, a, b[y]);
        }
      }
    }
  }

  using BFrag = V8[2][NP];

  // the B fragments of K step ks (both column tiles of the wave)
  static NTU_DEV void load_b(BFrag& b, const E* __restrict__ F, int ks, int w, int lane) {
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int p = 0; p < NP; ++p)
        b[y][p] = *(const V8*)(F + ((size_t)(((2 * w + y) * KS + ks) * NP + p) * 64 + lane) * 8);
  }

  // acc = A B^T with A from the shared pieces sA (NPAD rows, 2 NPAD real
  // columns) and B from prepared fragments F (layout of k_e45_prep); b0
  // holds the fragments of the first K step, loaded by the caller ahead of
  // time
  static NTU_DEV void product(Acc& acc, const E (*sA)[NPAD][LD], const E* __restrict__ F, int w, int lane,
                              const BFrag& b0) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      BFrag b;
      if (ks == 0) {
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int p = 0; p < NP; ++p) b[y][p] = b0[y][p];
      } else {
        load_b(b, F, ks, w, lane);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        V8 a[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) a[p] = *(const V8*)&sA[p][16 * mt + (lane & 15)][32 * ks + 8 * (lane >> 4)];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          if (ks == 0) mma<true>(acc, mt, y, a, b[y]);
          else mma<false>(acc, mt, y, a, b[y]);
        }
      }
    }
  }

  // Hands each complex output to fn(row, column, re, im), the accumulators
  // combined in FP32.
  template <class Fn> static NTU_DEV void outputs(const Acc& acc, int w, int lane, Fn fn) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        float x[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = comb(acc, mt, y, v);
        const int row = 16 * mt + (lane & 15);
        const int col = 16 * w + 8 * y + 2 * (lane >> 4);
        fn(row, col, x[0], x[1]);
        fn(row, col + 1, x[2], x[3]);
      }
  }

  // the same with both complex columns (col, col + 1) of a lane at once
  template <class Fn> static NTU_DEV void outputs4(const Acc& acc, int w, int lane, Fn fn) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        float x[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = comb(acc, mt, y, v);
        fn(16 * mt + (lane & 15), 16 * w + 8 * y + 2 * (lane >> 4), x);
      }
  }

  // pieces of the complex value (re, im) into row `row`, complex column colc
  static NTU_DEV void store_pieces(E (*sA)[NPAD][LD], int row, int colc, float re, float im) {
    unsigned t[NP];
    if constexpr (F16) split_pair_f16(re, im, t);
    else split_pair<PREC>(re, im, t);
#pragma unroll
    for (int p = 0; p < NP; ++p) *(unsigned*)&sA[p][row][2 * colc] = t[p];
  }
};

// Workgroups are dealt to the 8 XCDs round-robin by id; this order puts an
// item's workgroups on one XCD, consecutively.  The grid has 8 ceil(nwork / 8)
// workgroups; ids beyond the work return at once.
NTU_DEV int xcd_order(int nwork) {
  const int per = (nwork + 7) / 8;
  return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

// One workgroup per (item, a, a'): the Left block from the dressed
// isometries, then L1 and L2; the L2 block (FP32 (re, im) pairs, item stride
// hs complex elements, block (a R + a') n^2, row-major [j][k]) goes to out.
//   Left[b b'][t t'] = P[b D + t][b' D + t'],  P = QXe[a] QXp[a']^H
// FP16X3: every operand is scaled by a power of two into float16's range
// (the isometry blocks and each intermediate by their largest entry, EtopT /
// EbotT by the item scales of k_e45_scale); the L2 block is written as its
// two float16 pieces (row layout of k_mfma_tile_f16: per complex entry the
// packed hi word, then the lo word) scaled by a power of two, and that row's
// total scale goes to rowscale[item R^2 + a R + a'].
template <int PREC, int D, int NPAD = ((D * D + 15) / 16) * 16>
__global__ void __launch_bounds__(NPAD * 4, 2) k_left_e45(int R, int K, int nwork, const cd* __restrict__ QXe,
                                                       const cd* __restrict__ QXp, long long qs, float* __restrict__ out,
                                                       long long hs, const typename SplitTraits<PREC>::E* __restrict__ frag,
                                                       const float* __restrict__ escale, float* __restrict__ rowscale,
                                                       const float* __restrict__ blk) {
  using S = E45<PREC, NPAD>;
  using E = typename S::E;
  constexpr int NP = S::NP, LD = S::LD;
  constexpr bool F16 = S::F16;
  __shared__ __attribute__((aligned(16))) E sA[NP][NPAD][LD];
  __shared__ float red[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = xcd_order(nwork);
  if (q >= nwork) return;
  constexpr int n = D * D;
  const int R2 = R * R;
  const int item = q / R2, a = (q % R2) / R, ap = q % R;
  const cd* Qe = QXe + (size_t)item * qs + (size_t)a * n * K;
  const cd* Qp = QXp + (size_t)item * qs + (size_t)ap * n * K;
  const int per_m = e45_frag_elems(NPAD, NP);
  const E* F1 = frag + (size_t)item * 2 * per_m;
  const E* F2 = F1 + per_m;

  // zero the pieces when n < NPAD (rows and columns beyond n stay zero)
  if constexpr (n < NPAD)
    for (int e = tid; e < NP * NPAD * LD / 2; e += blockDim.x) ((unsigned*)&sA[0][0][0])[e] = 0u;
  typename S::Acc acc;
  typename S::BFrag b0;
  S::load_b(b0, F1, 0, w, lane);  // in flight during the Left block
  // FP16X3 scales; tot: the factor the values in acc carry
  float se = 1.0f, sp = 1.0f, tot = 1.0f, sn = 1.0f;
  if constexpr (F16) {
    se = blk[((size_t)item * 4 + 0) * R + a];
    sp = blk[((size_t)item * 4 + 1) * R + ap];
  }
  S::pair_product(acc, Qe, Qp, n, K, w, lane, se, sp);
  if constexpr (F16) {
    sn = S::acc_scale(acc, red);
    tot = se * sp * sn;
  }
  __syncthreads();
  S::outputs(acc, w, lane, [&](int u, int up, float re, float im) {
    if (u < n && up < n) S::store_pieces(sA, (u / D) * D + up / D, (u % D) * D + up % D, sn * re, sn * im);
  });
  __syncthreads();
  S::product(acc, sA, F1, w, lane, b0);
  S::load_b(b0, F2, 0, w, lane);  // in flight during the L1 hand-over
  if constexpr (F16) {
    sn = S::acc_scale(acc, red);
    tot *= escale[item * 2] * sn;
  }
  __syncthreads();  // every wave has read the Left pieces
  // L1 (row b b', column j) -> A operand of the second product: row j, column b b'
  S::outputs(acc, w, lane, [&](int bb, int j, float re, float im) { S::store_pieces(sA, j, bb, sn * re, sn * im); });
  __syncthreads();
  S::product(acc, sA, F2, w, lane, b0);
  float* O = out + ((size_t)item * hs + (size_t)(q % R2) * n * n) * 2;
  if constexpr (F16) {
    sn = S::acc_scale(acc, red);
    tot *= escale[item * 2 + 1] * sn;
    unsigned* Ow = (unsigned*)O;
    S::outputs(acc, w, lane, [&](int j, int k, float re, float im) {
      if (j < n && k < n) {
        unsigned t[2];
        split_pair_f16(sn * re, sn * im, t);
        *(uint2*)&Ow[2 * ((size_t)j * n + k)] = make_uint2(t[0], t[1]);
      }
    });
    if (tid == 0) rowscale[(size_t)item * R2 + q % R2] = tot;
  } else if constexpr (n % 2 == 0) {
    // columns come in even-odd pairs: one 16-byte store per pair (n even keeps it aligned)
    S::outputs4(acc, w, lane, [&](int j, int k, const float (&x)[4]) {
      if (j < n && k < n) *(float4*)&O[2 * ((size_t)j * n + k)] = make_float4(x[0], x[1], x[2], x[3]);
    });
  } else {
    S::outputs(acc, w, lane, [&](int j, int k, float re, float im) {
      if (j < n && k < n) *(float2*)&O[2 * ((size_t)j * n + k)] = make_float2(re, im);
    });
  }
}

// One workgroup per (item, B, B'):
//   Right[T T'][c c'] = P[c D + T][c' D + T'],  P = QYe[B] QYp[B']^H,
// staged in shared memory and written row-major (block (B R + B') n^2).
// FP16X3: the block is written as its float16 pieces (per complex entry the
// hi word, then the lo word) scaled by a power of two, the total scale in
// rowscale[item R^2 + B R + B'].
template <int PREC, int D, int NPAD = ((D * D + 15) / 16) * 16>
__global__ void __launch_bounds__(NPAD * 4, 2) k_right(int R, int K, int nwork, const cd* __restrict__ QYe,
                                                    const cd* __restrict__ QYp, long long qs, float* __restrict__ out,
                                                    long long hs, float* __restrict__ rowscale,
                                                    const float* __restrict__ blk) {
  using S = E45<PREC, NPAD>;
  __shared__ __attribute__((aligned(16))) float2 st[NPAD * NPAD];
  __shared__ float red[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = xcd_order(nwork);
  if (q >= nwork) return;
  constexpr int n = D * D;
  const int R2 = R * R;
  const int item = q / R2, b = (q % R2) / R, bp = q % R;
  const cd* Qe = QYe + (size_t)item * qs + (size_t)b * n * K;
  const cd* Qp = QYp + (size_t)item * qs + (size_t)bp * n * K;
  typename S::Acc acc;
  float se = 1.0f, sp = 1.0f, sn = 1.0f;
  if constexpr (S::F16) {
    se = blk[((size_t)item * 4 + 2) * R + b];
    sp = blk[((size_t)item * 4 + 3) * R + bp];
  }
  S::pair_product(acc, Qe, Qp, n, K, w, lane, se, sp);
  if constexpr (S::F16) sn = S::acc_scale(acc, red);
  S::outputs(acc, w, lane, [&](int u, int up, float re, float im) {
    if (u < n && up < n) st[((u % D) * D + up % D) * n + (u / D) * D + up / D] = make_float2(sn * re, sn * im);
  });
  __syncthreads();
  if constexpr (S::F16) {
    unsigned* Ow = (unsigned*)(out + ((size_t)item * hs + (size_t)(q % R2) * n * n) * 2);
    for (int e = tid; e < n * n; e += blockDim.x) {
      unsigned t[2];
      split_pair_f16(st[e].x, st[e].y, t);
      *(uint2*)&Ow[2 * (size_t)e] = make_uint2(t[0], t[1]);
    }
    if (tid == 0) rowscale[(size_t)item * R2 + q % R2] = se * sp * sn;
  } else {
    float2* O = (float2*)(out + ((size_t)item * hs + (size_t)(q % R2) * n * n) * 2);
    for (int e = tid; e < n * n; e += blockDim.x) O[e] = st[e];
  }
}

bool e45_supported(bool cplx, int precision, int D) {
  return cplx && (precision == NTU_PREC_BF16X3 || precision == NTU_PREC_BF16X6 || precision == NTU_PREC_FP16X3) &&
         D * D <= 64;
}

size_t e45_frag_bytes(int precision, int batch, int D) {
  const int np = precision == NTU_PREC_BF16X6 ? 3 : 2;
  return (size_t)batch * 2 * e45_frag_elems(e45_npad(D), np) * sizeof(__bf16);
}

// FP16X3 scales after the prepared fragments in H1: per item the two
// operand scales of EtopT / EbotT, then the row scales of L2 and of Right,
// then the scales of the isometry blocks
E45Scales e45_scales(void* H1, int precision, int batch, int D, int R) {
  E45Scales sc;
  float* base = (float*)((char*)H1 + ((e45_frag_bytes(precision, batch, D) + 255) / 256) * 256);
  sc.e = base;
  sc.left = base + 2 * (size_t)batch;
  sc.right = sc.left + (size_t)batch * R * R;
  sc.blk = sc.right + (size_t)batch * R * R;
  return sc;
}

size_t e45_scale_bytes(int batch, int R) {
  return (2 + 2 * (size_t)R * R + 4 * (size_t)R) * batch * sizeof(float) + 256;
}

template <int PREC, int D>
static void fused_launch(int batch, int p, int R, const cd* QXe, const cd* QXp, const cd* QYe, const cd* QYp,
                         long long qs, float* L2, float* Right, long long hs,
                         const typename SplitTraits<PREC>::E* frag, const E45Scales& sc, hipStream_t st,
                         const ProfHook& ph) {
  constexpr int NPAD = ((D * D + 15) / 16) * 16;
  const int nwork = batch * R * R;
  const dim3 g(8 * ((nwork + 7) / 8)), b(NPAD * 4);
  ph(PK_LEFTRIGHT, 0);
  if (PREC == NTU_PREC_FP16X3)
    hipLaunchKernelGGL(k_e45_blockscale, dim3(R, 4, batch), dim3(256), 0, st, D * D, p * D, R, QXe, QXp, QYe, QYp, qs,
                       sc.blk);
  hipLaunchKernelGGL((k_right<PREC, D>), g, b, 0, st, R, p * D, nwork, QYe, QYp, qs, Right, hs, sc.right, sc.blk);
  ph(PK_LEFTRIGHT, 1);
  ph(PK_E4, 0);
  hipLaunchKernelGGL((k_left_e45<PREC, D>), g, b, 0, st, R, p * D, nwork, QXe, QXp, qs, L2, hs, frag, sc.e,
                     sc.left, sc.blk);
  ph(PK_E4, 1);
}

template <int PREC>
static hipError_t fused_run(int batch, int p, int D, int R, const void* QXe, const void* QXp, const void* QYe,
                            const void* QYp, const void* ETT, const void* EBT, long long es, long long qs, void* H0,
                            void* H1, void* H2, long long hs, hipStream_t st, const ProfHook& ph) {
  using E = typename SplitTraits<PREC>::E;
  const int n = D * D, npad = e45_npad(D);
  constexpr int NP = SplitTraits<PREC>::NT;
  const int nval = e45_frag_elems(npad, NP) / NP;
  const E45Scales sc = e45_scales(H1, PREC, batch, D, R);
  ph(PK_E5, 0);
  if (PREC == NTU_PREC_FP16X3)
    hipLaunchKernelGGL(k_e45_scale, dim3(batch, 2), dim3(256), 0, st, n, (const cd*)ETT, (const cd*)EBT, es, sc.e);
  hipLaunchKernelGGL(k_e45_prep<PREC>, dim3((nval + 255) / 256, batch, 2), dim3(256), 0, st, n, npad,
                     (const cd*)ETT, (const cd*)EBT, es, (E*)H1, (const float*)sc.e);
  ph(PK_E5, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define NTU_FUSED(D_)                                                                                           \
  fused_launch<PREC, D_>(batch, p, R, (const cd*)QXe, (const cd*)QXp, (const cd*)QYe, (const cd*)QYp, qs, (float*)H0, \
                         (float*)H2, hs, (const E*)H1, sc, st, ph)
  switch (D) {
    case 1: NTU_FUSED(1); break;
    case 2: NTU_FUSED(2); break;
    case 3: NTU_FUSED(3); break;
    case 4: NTU_FUSED(4); break;
    case 5: NTU_FUSED(5); break;
    case 6: NTU_FUSED(6); break;
    case 7: NTU_FUSED(7); break;
    case 8: NTU_FUSED(8); break;
    default: return hipErrorInvalidValue;
  }
#undef NTU_FUSED
  return hipGetLastError();
}

hipError_t launch_env_fused(int precision, int batch, int p, int D, int R, const void* QXe, const void* QXp,
                            const void* QYe, const void* QYp, const void* ETT, const void* EBT, long long es,
                            long long qs, void* H0, void* H1, void* H2, long long hs, hipStream_t st,
                            const ProfHook& ph) {
  if (batch <= 0) return hipSuccess;
  if (D * D > 64) return hipErrorInvalidValue;
  if (e45_frag_bytes(precision, batch, D) + e45_scale_bytes(batch, R) + 256 > (size_t)batch * hs * 8)
    return hipErrorInvalidValue;
  if (precision == NTU_PREC_FP16X3)
    return fused_run<NTU_PREC_FP16X3>(batch, p, D, R, QXe, QXp, QYe, QYp, ETT, EBT, es, qs, H0, H1, H2, hs, st, ph);
  if (precision == NTU_PREC_BF16X6)
    return fused_run<NTU_PREC_BF16X6>(batch, p, D, R, QXe, QXp, QYe, QYp, ETT, EBT, es, qs, H0, H1, H2, hs, st, ph);
  if (precision == NTU_PREC_BF16X3)
    return fused_run<NTU_PREC_BF16X3>(batch, p, D, R, QXe, QXp, QYe, QYp, ETT, EBT, es, qs, H0, H1, H2, hs, st, ph);
  return hipErrorNotSupported;
}

}  // namespace ntu
