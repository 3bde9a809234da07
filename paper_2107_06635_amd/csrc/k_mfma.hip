// Split-precision NT products on the gfx950 matrix cores:
//   C(i, j) = sum_k A(i, k) B(j, k)
// Each operand value x is split into bfloat16 (or float16) pieces,
//   BF16X3:  x = hi + lo,          product ~ hi*hi + (hi*lo + lo*hi)
//   BF16X6:  x = hi + mid + lo,    product ~ hi*hi + (hi*mid + mid*hi)
//                                            + (hi*lo + mid*mid + lo*hi)
//   FP16X3:  x s = hi + lo 2^-11,  product ~ hi*hi + 2^-11 (hi*lo + lo*hi)
// with every term class accumulated in its own FP32 MFMA accumulator and the
// classes combined in FP64 at the end (split-K partials are summed in FP64).
// Complex operands use the real embedding: an interleaved complex row of A
// is a real row of length 2K; each complex row of B yields two real rows
// (re, -im), (im, re) (or (re, im), (-im, re) for conj(B)), so the real
// product has output columns (re, im) interleaved.
#include "kernels.h"
#include "mfma_gemm.h"
#include "split_mfma.h"

namespace ntu {

constexpr int MT_BM = 64, MT_BN = 64, MT_BK = 32, MT_PAD = 8, MT_LD = MT_BK + MT_PAD;

template <class TIn> NTU_DEV float to_f(TIn v) { return (float)v; }

// Load the real value (row, kr) of the real-embedded operand.
//  A-side (expand = false): real row i, real k -> element k of the (interleaved) row
//  B-side complex (expand = true): real row jr -> complex row jr/2, part jr%2
template <bool CPLX, bool EXPAND, class TIn>
NTU_DEV float load_real(const TIn* rowp, int jr_parity, int kr, int conj) {
  if constexpr (!CPLX || !EXPAND) {
    return to_f(rowp[kr]);
  } else {
    const int kc = kr >> 1, part = kr & 1;
    float re = to_f(rowp[2 * kc]), im = to_f(rowp[2 * kc + 1]);
    if (conj) im = -im;
    // row 2j (C_re): (re, -im) ; row 2j+1 (C_im): (im, re)
    if (jr_parity == 0) return part == 0 ? re : -im;
    return part == 0 ? im : re;
  }
}

struct MixedArgs {
  GemmNT d;          // in complex (or real) elements
  int ksplit;        // number of K chunks (grid.z = batch * ksplit)
  int kchunk;        // real K per chunk (multiple of MT_BK)
  double* partial;   // ksplit > 1: [split][item][M][Nr] FP64 partial sums
  const float* scaleA;  // FP16X3: per-item power-of-two scale of A (NULL = 1)
  const float* scaleB;
};

template <int PREC, bool CPLX, class TA, class TB, class TC>
__global__ void __launch_bounds__(256) k_mfma_nt(const TA* __restrict__ A, const TB* __restrict__ B,
                                                TC* __restrict__ C, MixedArgs args) {
  using E = typename SplitTraits<PREC>::E;
  constexpr int NT = SplitTraits<PREC>::NT;
  constexpr int NACC = (PREC == NTU_PREC_BF16X6) ? 3 : 2;
  __shared__ __attribute__((aligned(16))) E sA[NT][MT_BM][MT_LD];
  __shared__ __attribute__((aligned(16))) E sB[NT][MT_BN][MT_LD];
  const GemmNT& d = args.d;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int Mr = d.M, Nr = CPLX ? 2 * d.N : d.N, Kr = CPLX ? 2 * d.K : d.K;
  const int item = blockIdx.z / args.ksplit, split = blockIdx.z % args.ksplit;
  const int i0 = blockIdx.y * MT_BM, j0 = blockIdx.x * MT_BN;
  const int kbeg = split * args.kchunk;
  const int kend = min(Kr, kbeg + args.kchunk);
  constexpr int CW = CPLX ? 2 : 1;  // scalars per element
  const TA* Ab = A + idx_off(d.Ab, item) * CW;
  const TB* Bb = B + idx_off(d.Bb, item) * CW;
  float scA = 1.0f, scB = 1.0f;
  if constexpr (PREC == NTU_PREC_FP16X3) {
    if (args.scaleA) scA = args.scaleA[item];
    if (args.scaleB) scB = args.scaleB[item];
  }
  // each thread stages 8 consecutive real k of one tile row
  const int lrow = tid >> 2, lk = (tid & 3) * 8;
  const int ai = i0 + lrow, bj = j0 + lrow;
  const TA* arow = ai < Mr ? Ab + idx_off(d.Ai, ai) * CW : nullptr;
  const int bcol = CPLX ? (bj >> 1) : bj;
  const TB* brow = bj < Nr ? Bb + idx_off(d.Bj, bcol) * CW : nullptr;

  f32x4 acc[NACC][2][2];
#pragma unroll
  for (int c = 0; c < NACC; ++c)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[c][x][y] = f32x4{0, 0, 0, 0};

  for (int k0 = kbeg; k0 < kend; k0 += MT_BK) {
    E pa[NT][8], pb[NT][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int kr = k0 + lk + u;
      float va = 0.0f, vb = 0.0f;
      if (kr < kend) {
        if (arow) va = load_real<CPLX, false>(arow, 0, kr, 0) * scA;
        if (brow) vb = load_real<CPLX, true>(brow, bj & 1, kr, d.conjB) * scB;
      }
      E ta[NT], tb[NT];
      split_value<PREC>(va, ta);
      split_value<PREC>(vb, tb);
#pragma unroll
      for (int t = 0; t < NT; ++t) { pa[t][u] = ta[t]; pb[t][u] = tb[t]; }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        sA[t][lrow][lk + u] = pa[t][u];
        sB[t][lrow][lk + u] = pb[t][u];
      }
    }
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int ra = wm * 32 + x * 16 + fr, rb = wn * 32 + y * 16 + fr;
        const E* a0 = &sA[0][ra][fk];
        const E* b0 = &sB[0][rb][fk];
        const E* a1 = &sA[1][ra][fk];
        const E* b1 = &sB[1][rb][fk];
        acc[0][x][y] = mfma<PREC>(a0, b0, acc[0][x][y]);
        acc[1][x][y] = mfma<PREC>(a0, b1, acc[1][x][y]);
        acc[1][x][y] = mfma<PREC>(a1, b0, acc[1][x][y]);
        if constexpr (PREC == NTU_PREC_BF16X6) {
          const E* a2 = &sA[2][ra][fk];
          const E* b2 = &sB[2][rb][fk];
          acc[2][x][y] = mfma<PREC>(a0, b2, acc[2][x][y]);
          acc[2][x][y] = mfma<PREC>(a1, b1, acc[2][x][y]);
          acc[2][x][y] = mfma<PREC>(a2, b0, acc[2][x][y]);
        }
      }
    }
  }
  // epilogue: output layout of the 16x16 result: lane holds column (lane & 15),
  // rows 4 * (lane >> 4) + v
  const double unscale = 1.0 / ((double)scA * (double)scB);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wm * 32 + x * 16 + 4 * (lane >> 4) + v;
        const int jr = j0 + wn * 32 + y * 16 + (lane & 15);
        if (i >= Mr || jr >= Nr) continue;
        double val;
        if constexpr (PREC == NTU_PREC_FP16X3) val = ((double)acc[0][x][y][v] + (double)acc[1][x][y][v] * (1.0 / 2048.0)) * unscale;
        else if constexpr (PREC == NTU_PREC_BF16X6) val = (double)acc[0][x][y][v] + ((double)acc[1][x][y][v] + (double)acc[2][x][y][v]);
        else val = (double)acc[0][x][y][v] + (double)acc[1][x][y][v];
        if (args.ksplit > 1) {
          args.partial[(((size_t)split * d.batch + item) * Mr + i) * Nr + jr] = val;
        } else {
          const int j = CPLX ? jr >> 1 : jr, part = CPLX ? jr & 1 : 0;
          long long off = (idx_off(d.Cb, item) + idx_off(d.Ci, i) + idx_off(d.Cj, j)) * CW + part;
          C[off] = (TC)val;
        }
      }
}

// ---------------------------------------------------------------------------
// Tiled variant for operands whose rows are contiguous in K (all products of
// the environment contraction): 128 x 128 real-embedded output tiles, eight
// waves of 64 x 32 (4 x 2 MFMA tiles each), K in steps of 32 with the next
// step's global loads in registers while the current step runs on the
// matrix cores, double-buffered shared memory, one barrier per step.
// Blocks are dealt to the 8 XCDs round-robin by id; the tile order puts the
// tiles (and K chunks) of one item on one XCD, consecutively, so they share
// that XCD's L2.  Output offsets are tabulated once per block.  Eight waves
// (two per SIMD) so that one wave's matrix-core work overlaps another's
// operand staging.
// VEC = 2: pairs of values per load (K and all row strides even).
// ---------------------------------------------------------------------------
constexpr int TL_M = 128, TL_N = 128, TL_K = 32, TL_LD = TL_K;
constexpr int TL_THREADS = 512, TL_WY = 2;  // 8 waves; each 64 x (16 TL_WY)
// the FP16X3 assembly from pre-split operands: each wave 64 x (16 F16_WY)
constexpr int F16_WY = 2;

// Shared-memory layout of an operand tile: unpadded rows of TL_K pieces (64
// bytes, a quarter of the 64 four-byte banks), the four 16-byte chunks of row
// r permuted by chunk ^ ((r >> 1) & 3).  The matrix-core reads (16-byte
// chunks, lanes 0-7 with 16-23 served together, and so on) then meet each
// bank once, and so do the 8-byte stores of four consecutive rows.
NTU_DEV int tl_col(int row, int k) { return (((k >> 3) ^ ((row >> 1) & 3)) << 3) | (k & 7); }

struct alignas(8) f2v { float v[2]; };
struct alignas(16) d2v { double v[2]; };
template <int VEC, class TIn> NTU_DEV void load_pair(const TIn* p, float* out);
template <> NTU_DEV void load_pair<2, float>(const float* p, float* out) {
  const f2v x = *(const f2v*)p;
  out[0] = x.v[0]; out[1] = x.v[1];
}
template <> NTU_DEV void load_pair<2, double>(const double* p, float* out) {
  const d2v x = *(const d2v*)p;
  out[0] = (float)x.v[0]; out[1] = (float)x.v[1];
}

struct TileArgs {
  GemmNT d;
  int tiles_m, tiles_n, ksplit, kchunk;  // kchunk: real K per chunk, multiple of TL_K
  int nwork;                             // batch * tiles * ksplit
  double* partial;                       // ksplit > 1: [split][item][Mr][Nr]
};

template <int PREC, bool CPLX, int VEC, class TA, class TB, class TC>
__global__ void __launch_bounds__(TL_THREADS) k_mfma_tile(const TA* __restrict__ A, const TB* __restrict__ B,
                                                  TC* __restrict__ C, TileArgs ta) {
  using E = typename SplitTraits<PREC>::E;
  constexpr int NT = SplitTraits<PREC>::NT;
  constexpr int NACC = (PREC == NTU_PREC_BF16X6) ? 3 : 2;
  constexpr int CW = CPLX ? 2 : 1;
  constexpr int NGA = TL_M * TL_K / 4 / TL_THREADS;          // groups of 4 reals of A per thread
  constexpr int NGB = CPLX ? NGA / 2 : NGA;                  // of B (complex rows give two real rows)
  // one buffer for both operands (double-buffered); the output tile of a
  // 4-byte result (rows of TL_N + 1) reuses it
  constexpr int SA_EL = 2 * NT * TL_M * TL_LD, SB_EL = 2 * NT * TL_N * TL_LD;
  constexpr int OUT_EL = sizeof(TC) == 4 ? (int)(TL_M * (TL_N + 1) * sizeof(TC) / sizeof(E)) : 0;
  constexpr int SM_EL = SA_EL + SB_EL > OUT_EL ? SA_EL + SB_EL : OUT_EL;
  __shared__ __attribute__((aligned(16))) E smem[SM_EL];
  E (*sA)[NT][TL_M][TL_LD] = reinterpret_cast<E (*)[NT][TL_M][TL_LD]>(smem);
  E (*sB)[NT][TL_N][TL_LD] = reinterpret_cast<E (*)[NT][TL_N][TL_LD]>(smem + SA_EL);
  __shared__ long long rowoff[TL_M];
  __shared__ long long coloff[TL_N];
  const GemmNT& d = ta.d;
  // 8 waves: 2 along M (64 rows each) x 4 along N (32 columns each)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 2, wn = wv & 3;
  const int per = (ta.nwork + 7) / 8;
  const int q = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (q >= ta.nwork) return;
  const int T = ta.tiles_m * ta.tiles_n;
  const int item = q / (T * ta.ksplit), rem = q % (T * ta.ksplit);
  const int tile = rem / ta.ksplit, split = rem % ta.ksplit;
  const int i0 = (tile / ta.tiles_n) * TL_M, j0 = (tile % ta.tiles_n) * TL_N;
  const int Mr = d.M, Nr = CW * d.N, Kr = CW * d.K;
  const int kbeg = split * ta.kchunk, kend = min(Kr, kbeg + ta.kchunk);
  const TA* Ab = A + idx_off(d.Ab, item) * CW;
  const TB* Bb = B + idx_off(d.Bb, item) * CW;

  for (int r = tid; r < TL_M; r += TL_THREADS) {
    const int i = i0 + r;
    rowoff[r] = i < Mr ? idx_off(d.Ci, i) * CW : -1;
  }
  for (int c = tid; c < TL_N; c += TL_THREADS) {
    const int jr = j0 + c;
    coloff[c] = jr < Nr ? idx_off(d.Cj, CPLX ? jr >> 1 : jr) * CW + (CPLX ? (jr & 1) : 0) : -1;
  }
  // this thread's load groups: (row, 4 reals at kq)
  const TA* arow[NGA];
  int akq[NGA], arl[NGA];
#pragma unroll
  for (int u = 0; u < NGA; ++u) {
    const int g = tid + TL_THREADS * u, rl = g / (TL_K / 4);
    arl[u] = rl;
    akq[u] = (g % (TL_K / 4)) * 4;
    arow[u] = i0 + rl < Mr ? Ab + idx_off(d.Ai, i0 + rl) * CW : nullptr;
  }
  const TB* brow[NGB];
  int bkq[NGB], brl[NGB];
#pragma unroll
  for (int u = 0; u < NGB; ++u) {
    const int g = tid + TL_THREADS * u, rl = g / (TL_K / 4);   // rl: complex row (CPLX) or real row
    brl[u] = rl;
    bkq[u] = (g % (TL_K / 4)) * 4;
    const int jrow = CPLX ? j0 / 2 + rl : j0 + rl;
    const bool ok = CPLX ? 2 * jrow < Nr : jrow < Nr;
    brow[u] = ok ? Bb + idx_off(d.Bj, jrow) * CW : nullptr;
  }
  // two register sets of operand values: the loads of step s + 2 are in
  // flight while step s runs and step s + 1's values are split and stored.
  // The loads are unconditional (a missing row reads the item's first row, a
  // value beyond the chunk the chunk's first column, always in bounds) and
  // the values that do not exist are zeroed when stored: loads under a
  // branch would each wait for their data at the join.
  float ra0[NGA][4], rb0[NGB][4], ra1[NGA][4], rb1[NGB][4];
  unsigned oka0[NGA], okb0[NGB], oka1[NGA], okb1[NGB];  // bit e: value e exists
  auto ld4 = [&](const auto* row, const auto* base, int k, float (&r)[4], unsigned& ok) {
    const auto* p = row ? row : base;
    ok = 0u;
    if constexpr (VEC == 2) {
      const bool o0 = row && k < kend, o1 = row && k + 2 < kend;
      load_pair<2>(p + (o0 ? k : kbeg), &r[0]);
      load_pair<2>(p + (o1 ? k + 2 : kbeg), &r[2]);
      ok = (o0 ? 3u : 0u) | (o1 ? 12u : 0u);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool o = row && k + e < kend;
        r[e] = (float)p[o ? k + e : kbeg];
        ok |= o ? (1u << e) : 0u;
      }
    }
  };
  auto gload = [&](int k0, float (&ra)[NGA][4], float (&rb)[NGB][4], unsigned (&oka)[NGA], unsigned (&okb)[NGB]) {
#pragma unroll
    for (int u = 0; u < NGA; ++u) ld4(arow[u], Ab, k0 + akq[u], ra[u], oka[u]);
#pragma unroll
    for (int u = 0; u < NGB; ++u) ld4(brow[u], Bb, k0 + bkq[u], rb[u], okb[u]);
  };
  // zero the values that do not exist (in a copy, at store time)
  auto masked = [](const float (&r)[4], unsigned ok, float (&o)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = (ok >> e) & 1u ? r[e] : 0.0f;
  };
  auto lstore = [&](int buf, const float (&ra_in)[NGA][4], const float (&rb_in)[NGB][4], const unsigned (&oka)[NGA],
                    const unsigned (&okb)[NGB]) {
    float ra[NGA][4], rb[NGB][4];
#pragma unroll
    for (int u = 0; u < NGA; ++u) masked(ra_in[u], oka[u], ra[u]);
#pragma unroll
    for (int u = 0; u < NGB; ++u) masked(rb_in[u], okb[u], rb[u]);
    if constexpr (PREC != NTU_PREC_FP16X3) {
      // bfloat16 pieces of two values at once (one packed word per piece)
#pragma unroll
      for (int u = 0; u < NGA; ++u) {
        unsigned w0[NT], w1[NT];
        split_pair<PREC>(ra[u][0], ra[u][1], w0);
        split_pair<PREC>(ra[u][2], ra[u][3], w1);
#pragma unroll
        for (int p = 0; p < NT; ++p) *(uint2*)&sA[buf][p][arl[u]][tl_col(arl[u], akq[u])] = make_uint2(w0[p], w1[p]);
      }
#pragma unroll
      for (int u = 0; u < NGB; ++u) {
        if constexpr (CPLX) {
          // complex values (re0, im0), (re1, im1) -> real rows 2r: (re, -im), 2r+1: (im, re).
          // The pieces of (re, im) are split once; the pieces of -x are those
          // of x negated (sign bit), so row 2r flips the high halves and row
          // 2r+1 swaps the halves.  Complex rows 0, 1, 2, 3 store real rows
          // 0, 3, 5, 6 first (one row per bank quarter), then 1, 2, 4, 7.
          const float s = d.conjB ? -1.0f : 1.0f;
          unsigned w0[NT], w1[NT];
          split_pair<PREC>(rb[u][0], s * rb[u][1], w0);
          split_pair<PREC>(rb[u][2], s * rb[u][3], w1);
          const int odd_first = (brl[u] ^ (brl[u] >> 1)) & 1;
          const int r0 = 2 * brl[u] + odd_first, r1 = 2 * brl[u] + 1 - odd_first;
          const int c0 = tl_col(r0, bkq[u]), c1 = tl_col(r1, bkq[u]);
#pragma unroll
          for (int p = 0; p < NT; ++p) {
            const uint2 neg = make_uint2(w0[p] ^ 0x80000000u, w1[p] ^ 0x80000000u);
            const uint2 swp = make_uint2((w0[p] >> 16) | (w0[p] << 16), (w1[p] >> 16) | (w1[p] << 16));
            *(uint2*)&sB[buf][p][r0][c0] = odd_first ? swp : neg;
            *(uint2*)&sB[buf][p][r1][c1] = odd_first ? neg : swp;
          }
        } else {
          unsigned w0[NT], w1[NT];
          split_pair<PREC>(rb[u][0], rb[u][1], w0);
          split_pair<PREC>(rb[u][2], rb[u][3], w1);
#pragma unroll
          for (int p = 0; p < NT; ++p) *(uint2*)&sB[buf][p][brl[u]][tl_col(brl[u], bkq[u])] = make_uint2(w0[p], w1[p]);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < NGA; ++u) {
        E t[4][NT];
#pragma unroll
        for (int e = 0; e < 4; ++e) split_value<PREC>(ra[u][e], t[e]);
#pragma unroll
        for (int p = 0; p < NT; ++p)
#pragma unroll
          for (int e = 0; e < 4; ++e) sA[buf][p][arl[u]][tl_col(arl[u], akq[u]) + e] = t[e][p];
      }
#pragma unroll
      for (int u = 0; u < NGB; ++u) {
        if constexpr (CPLX) {
          // complex values (re0, im0), (re1, im1) -> real rows 2r: (re, -im), 2r+1: (im, re)
          const float s = d.conjB ? -1.0f : 1.0f;
          const float re0 = rb[u][0], im0 = s * rb[u][1], re1 = rb[u][2], im1 = s * rb[u][3];
          const float v0[4] = {re0, -im0, re1, -im1}, v1[4] = {im0, re0, im1, re1};
          E t0[4][NT], t1[4][NT];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            split_value<PREC>(v0[e], t0[e]);
            split_value<PREC>(v1[e], t1[e]);
          }
#pragma unroll
          for (int p = 0; p < NT; ++p)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              sB[buf][p][2 * brl[u]][tl_col(2 * brl[u], bkq[u]) + e] = t0[e][p];
              sB[buf][p][2 * brl[u] + 1][tl_col(2 * brl[u] + 1, bkq[u]) + e] = t1[e][p];
            }
        } else {
          E t[4][NT];
#pragma unroll
          for (int e = 0; e < 4; ++e) split_value<PREC>(rb[u][e], t[e]);
#pragma unroll
          for (int p = 0; p < NT; ++p)
#pragma unroll
            for (int e = 0; e < 4; ++e) sB[buf][p][brl[u]][tl_col(brl[u], bkq[u]) + e] = t[e][p];
        }
      }
    }
  };


  f32x4 acc[NACC][4][TL_WY];
#pragma unroll
  for (int c = 0; c < NACC; ++c)
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < TL_WY; ++y) acc[c][x][y] = f32x4{0, 0, 0, 0};

  // an even number of steps, every load and store unconditional (see above):
  // a step beyond the chunk adds zero products
  const int nsteps = (((kend - kbeg + TL_K - 1) / TL_K) + 1) & ~1;
  gload(kbeg, ra0, rb0, oka0, okb0);
  lstore(0, ra0, rb0, oka0, okb0);
  gload(kbeg + TL_K, ra1, rb1, oka1, okb1);
  __syncthreads();
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  // the 16-byte chunk this lane reads from each of its rows (tile rows are
  // multiples of 16 plus fr, so the permutation depends on fr alone)
  const int fks = tl_col(fr, fk);
  auto products = [&](int buf) {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int ra_ = wm * 64 + x * 16 + fr;
#pragma unroll
      for (int y = 0; y < TL_WY; ++y) {
        const int rb_ = wn * (16 * TL_WY) + y * 16 + fr;
        const E* a0 = &sA[buf][0][ra_][fks];
        const E* a1 = &sA[buf][1][ra_][fks];
        const E* b0 = &sB[buf][0][rb_][fks];
        const E* b1 = &sB[buf][1][rb_][fks];
        acc[0][x][y] = mfma<PREC>(a0, b0, acc[0][x][y]);
        acc[1][x][y] = mfma<PREC>(a0, b1, acc[1][x][y]);
        acc[1][x][y] = mfma<PREC>(a1, b0, acc[1][x][y]);
        if constexpr (PREC == NTU_PREC_BF16X6) {
          const E* a2 = &sA[buf][2][ra_][fks];
          const E* b2 = &sB[buf][2][rb_][fks];
          acc[2][x][y] = mfma<PREC>(a0, b2, acc[2][x][y]);
          acc[2][x][y] = mfma<PREC>(a1, b1, acc[2][x][y]);
          acc[2][x][y] = mfma<PREC>(a2, b0, acc[2][x][y]);
        }
      }
    }
  };
  for (int s = 0; s < nsteps; s += 2) {
    gload(kbeg + (s + 2) * TL_K, ra0, rb0, oka0, okb0);
    products(0);
    lstore(1, ra1, rb1, oka1, okb1);
    __syncthreads();
    gload(kbeg + (s + 3) * TL_K, ra1, rb1, oka1, okb1);
    products(1);
    lstore(0, ra0, rb0, oka0, okb0);
    __syncthreads();
  }
  // epilogue: lane holds column (lane & 15), rows 4 (lane >> 4) + v of each 16 x 16 tile
  const long long cbase = idx_off(d.Cb, item) * CW;
  if constexpr (sizeof(TC) == 4) {
    if (ta.ksplit == 1) {
      // stage the tile in shared memory (the operand buffers are free after the
      // last barrier), then write it in the order that is contiguous in C:
      // row-major if consecutive real columns are adjacent, else column-major
      // (complex: (re, im) of consecutive rows adjacent)
      constexpr int OLD = TL_N + 1;
      static_assert(TL_M * OLD * sizeof(TC) <= SM_EL * sizeof(E), "output tile must fit the shared buffer");
      TC* ot = (TC*)smem;
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < TL_WY; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int il = wm * 64 + x * 16 + 4 * (lane >> 4) + v;
            const int jl = wn * (16 * TL_WY) + y * 16 + (lane & 15);
            double val;
            if constexpr (PREC == NTU_PREC_BF16X6) val = (double)acc[0][x][y][v] + ((double)acc[1][x][y][v] + (double)acc[2][x][y][v]);
            else val = (double)acc[0][x][y][v] + (double)acc[1][x][y][v];
            ot[il * OLD + jl] = (TC)val;
          }
      __syncthreads();
      const bool rowmajor = coloff[1] - coloff[0] == 1;
      for (int e = tid; e < TL_M * TL_N; e += TL_THREADS) {
        int il, jl;
        if (rowmajor) {
          il = e / TL_N;
          jl = e % TL_N;
        } else if (CPLX) {
          const int part = e & 1, t = e >> 1;
          il = t % TL_M;
          jl = 2 * (t / TL_M) + part;
        } else {
          il = e % TL_M;
          jl = e / TL_M;
        }
        const long long ro = rowoff[il], co = coloff[jl];
        if (ro >= 0 && co >= 0) C[cbase + ro + co] = ot[il * OLD + jl];
      }
      return;
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < TL_WY; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int il = wm * 64 + x * 16 + 4 * (lane >> 4) + v;
        const int jl = wn * (16 * TL_WY) + y * 16 + (lane & 15);
        double val;
        if constexpr (PREC == NTU_PREC_BF16X6) val = (double)acc[0][x][y][v] + ((double)acc[1][x][y][v] + (double)acc[2][x][y][v]);
        else val = (double)acc[0][x][y][v] + (double)acc[1][x][y][v];
        if (ta.ksplit > 1) {
          const int i = i0 + il, jr = j0 + jl;
          if (i < Mr && jr < Nr) ta.partial[(((size_t)split * d.batch + item) * Mr + i) * Nr + jr] = val;
        } else {
          const long long ro = rowoff[il], co = coloff[jl];
          if (ro >= 0 && co >= 0) C[cbase + ro + co] = (TC)val;
        }
      }
}

// ---------------------------------------------------------------------------
// The final assembly g = L2 Right^T in FP16X3 from operands the fused kernels
// wrote already split: each complex entry of a row is two packed words, the
// float16 hi pieces (re, im) then the lo pieces, the row scaled by its power
// of two (rows of A: sA[item][i], of B: sB[item][j]).  The
// K loop only moves pieces: global -> registers -> shared memory (complex B
// rows expanded to the two real rows (re, -im), (im, re) by a sign flip and a
// half swap of the packed words) -> MFMA.  Same tiling, buffering and block
// order as k_mfma_tile; C(i, j) = (hh + 2^-11 (hl + lh)) / (sA[i] sB[j]).
// ---------------------------------------------------------------------------
struct TileF16Args {
  int M, N, Kc, batch;          // rows of A and of B, complex K
  long long a_item, b_item;     // item strides (words) of A and B
  long long a_row, b_row;       // row strides (words): 2 Kc for contiguous rows
  const float* sA;              // [item][M]
  const float* sB;              // [item][N]
  Idx3 Cb, Ci, Cj;              // output maps (complex elements)
  int tiles_m, tiles_n, ksplit, kchunk;  // kchunk: real K per chunk
  int nwork;
  double* partial;              // ksplit > 1: [split][item][M][2N]
};

template <class TC, int WY>
__global__ void __launch_bounds__(TL_THREADS) k_mfma_tile_f16(const unsigned* __restrict__ A,
                                                              const unsigned* __restrict__ B, TC* __restrict__ C,
                                                              TileF16Args ta) {
  using E = _Float16;
  constexpr int NT = 2;
  constexpr int NGA = TL_M * TL_K / 4 / TL_THREADS;  // groups of 4 reals (2 complex) of A per thread
  constexpr int TN = 64 * WY;                        // columns of the tile: four waves of 16 WY
  constexpr int NGB = TN / 2 * TL_K / 4 / TL_THREADS;  // of B (each complex row gives two real rows)
  constexpr int SA_EL = 2 * NT * TL_M * TL_LD, SB_EL = 2 * NT * TN * TL_LD;
  __shared__ __attribute__((aligned(16))) E smem[SA_EL + SB_EL];
  E (*sA)[NT][TL_M][TL_LD] = reinterpret_cast<E (*)[NT][TL_M][TL_LD]>(smem);
  E (*sB)[NT][TN][TL_LD] = reinterpret_cast<E (*)[NT][TN][TL_LD]>(smem + SA_EL);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 2, wn = wv & 3;
  const int per = (ta.nwork + 7) / 8;
  const int q = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (q >= ta.nwork) return;
  const int T = ta.tiles_m * ta.tiles_n;
  const int item = q / (T * ta.ksplit), rem = q % (T * ta.ksplit);
  const int tile = rem / ta.ksplit, split = rem % ta.ksplit;
  const int i0 = (tile / ta.tiles_n) * TL_M, j0 = (tile % ta.tiles_n) * TN;
  const int Mr = ta.M, Nr = 2 * ta.N, Kr = 2 * ta.Kc;
  const int kbeg = split * ta.kchunk, kend = min(Kr, kbeg + ta.kchunk);
  const unsigned* Ab = A + (size_t)item * ta.a_item;
  const unsigned* Bb = B + (size_t)item * ta.b_item;
  // this thread's load groups: A row, 4 reals (2 words per piece) at real kq
  const unsigned* arow[NGA];
  int akq[NGA], arl[NGA];
#pragma unroll
  for (int u = 0; u < NGA; ++u) {
    const int g = tid + TL_THREADS * u, rl = g / (TL_K / 4);
    arl[u] = rl;
    akq[u] = (g % (TL_K / 4)) * 4;
    arow[u] = i0 + rl < Mr ? Ab + (size_t)(i0 + rl) * ta.a_row : nullptr;
  }
  const unsigned* brow[NGB];
  int bkq[NGB], brl[NGB];
#pragma unroll
  for (int u = 0; u < NGB; ++u) {
    const int g = tid + TL_THREADS * u, rl = g / (TL_K / 4);  // complex row
    brl[u] = rl;
    bkq[u] = (g % (TL_K / 4)) * 4;
    const int jrow = j0 / 2 + rl;
    brow[u] = 2 * jrow < Nr ? Bb + (size_t)jrow * ta.b_row : nullptr;
  }
  // registers: per group and piece, the two packed words (2 complex)
  uint2 ra0[NGA][NT], rb0[NGB][NT], ra1[NGA][NT], rb1[NGB][NT];
  // complex entries k / 2 and k / 2 + 1 (words k .. k + 3, each entry an
  // 8-byte aligned (hi, lo) pair; rows of odd length K end after the first).
  // The registers keep the loaded pairs as they are: regrouping them into
  // (hi, hi), (lo, lo) here would make the load wait at once; lstore
  // regroups, when the values are due.
  // The loads are unconditional (a missing row or an entry beyond the chunk
  // reads the row start or the first entry of the chunk instead, always in
  // bounds) and the entries that do not exist are zeroed when stored:
  // loads under a branch would each wait for their data at the join.
  auto ld2 = [&](const unsigned* row, const unsigned* base, int k, uint2 (&r)[NT], unsigned& ok) {
    const unsigned* p = row ? row : base;
    const bool ok0 = row && k < kend, ok1 = row && k + 2 < kend;
    r[0] = *(const uint2*)(p + (ok0 ? k : kbeg));
    r[1] = *(const uint2*)(p + (ok1 ? k + 2 : kbeg));
    ok = (ok0 ? 1u : 0u) | (ok1 ? 2u : 0u);
  };
  unsigned oka0[NGA], okb0[NGB], oka1[NGA], okb1[NGB];
  auto gload = [&](int k0, uint2 (&ra)[NGA][NT], uint2 (&rb)[NGB][NT], unsigned (&oka)[NGA],
                   unsigned (&okb)[NGB]) {
#pragma unroll
    for (int u = 0; u < NGA; ++u) ld2(arow[u], Ab, k0 + akq[u], ra[u], oka[u]);
#pragma unroll
    for (int u = 0; u < NGB; ++u) ld2(brow[u], Bb, k0 + bkq[u], rb[u], okb[u]);
  };
  // piece p of the two entries: (entry 0, entry 1) words of that piece, zero
  // where the entry does not exist
  auto piece = [](const uint2 (&r)[NT], int p, unsigned ok) {
    const unsigned w0 = p == 0 ? r[0].x : r[0].y, w1 = p == 0 ? r[1].x : r[1].y;
    return make_uint2((ok & 1u) ? w0 : 0u, (ok & 2u) ? w1 : 0u);
  };
  auto lstore = [&](int buf, const uint2 (&ra)[NGA][NT], const uint2 (&rb)[NGB][NT], const unsigned (&oka)[NGA],
                    const unsigned (&okb)[NGB]) {
#pragma unroll
    for (int u = 0; u < NGA; ++u)
#pragma unroll
      for (int p = 0; p < NT; ++p) *(uint2*)&sA[buf][p][arl[u]][tl_col(arl[u], akq[u])] = piece(ra[u], p, oka[u]);
#pragma unroll
    for (int u = 0; u < NGB; ++u) {
      // complex values (re0, im0), (re1, im1) -> real rows 2r: (re, -im),
      // 2r+1: (im, re); rows stored in bank-quarter order as in k_mfma_tile
      const int odd_first = (brl[u] ^ (brl[u] >> 1)) & 1;
      const int r0 = 2 * brl[u] + odd_first, r1 = 2 * brl[u] + 1 - odd_first;
      const int c0 = tl_col(r0, bkq[u]), c1 = tl_col(r1, bkq[u]);
#pragma unroll
      for (int p = 0; p < NT; ++p) {
        const uint2 w = piece(rb[u], p, okb[u]);
        const uint2 neg = make_uint2(w.x ^ 0x80000000u, w.y ^ 0x80000000u);
        const uint2 swp = make_uint2((w.x >> 16) | (w.x << 16), (w.y >> 16) | (w.y << 16));
        *(uint2*)&sB[buf][p][r0][c0] = odd_first ? swp : neg;
        *(uint2*)&sB[buf][p][r1][c1] = odd_first ? neg : swp;
      }
    }
  };

  f32x4 acc[2][4][WY];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < WY; ++y) acc[c][x][y] = f32x4{0, 0, 0, 0};

  // An even number of steps, every load and store unconditional: a step
  // beyond the chunk loads clamped addresses whose values are zeroed, and
  // adds zero products.  Without branches around them, the loads of step
  // s + 2 stay in flight while step s runs and step s + 1 is stored.
  const int nsteps = (((kend - kbeg + TL_K - 1) / TL_K) + 1) & ~1;
  gload(kbeg, ra0, rb0, oka0, okb0);
  lstore(0, ra0, rb0, oka0, okb0);
  gload(kbeg + TL_K, ra1, rb1, oka1, okb1);
  __syncthreads();
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  const int fks = tl_col(fr, fk);
  auto products = [&](int buf) {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int ra_ = wm * 64 + x * 16 + fr;
#pragma unroll
      for (int y = 0; y < WY; ++y) {
        const int rb_ = wn * (16 * WY) + y * 16 + fr;
        const E* a0 = &sA[buf][0][ra_][fks];
        const E* a1 = &sA[buf][1][ra_][fks];
        const E* b0 = &sB[buf][0][rb_][fks];
        const E* b1 = &sB[buf][1][rb_][fks];
        acc[0][x][y] = mfma<NTU_PREC_FP16X3>(a0, b0, acc[0][x][y]);
        acc[1][x][y] = mfma<NTU_PREC_FP16X3>(a0, b1, acc[1][x][y]);
        acc[1][x][y] = mfma<NTU_PREC_FP16X3>(a1, b0, acc[1][x][y]);
      }
    }
  };
  for (int s = 0; s < nsteps; s += 2) {
    gload(kbeg + (s + 2) * TL_K, ra0, rb0, oka0, okb0);
    products(0);
    lstore(1, ra1, rb1, oka1, okb1);
    __syncthreads();
    gload(kbeg + (s + 3) * TL_K, ra1, rb1, oka1, okb1);
    products(1);
    lstore(0, ra0, rb0, oka0, okb0);
    __syncthreads();
  }
  // epilogue: lane holds column (lane & 15), rows 4 (lane >> 4) + v of each 16 x 16 tile
  const float* sAi = ta.sA + (size_t)item * ta.M;
  const float* sBi = ta.sB + (size_t)item * ta.N;
  const long long cbase = idx_off(ta.Cb, item) * 2;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < WY; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wm * 64 + x * 16 + 4 * (lane >> 4) + v;
        const int jr = j0 + wn * (16 * WY) + y * 16 + (lane & 15);
        if (i >= Mr || jr >= Nr) continue;
        const double un = 1.0 / ((double)sAi[i] * (double)sBi[jr >> 1]);
        const double val = ((double)acc[0][x][y][v] + (double)acc[1][x][y][v] * (1.0 / 2048.0)) * un;
        if (ta.ksplit > 1) {
          ta.partial[(((size_t)split * ta.batch + item) * Mr + i) * Nr + jr] = val;
        } else {
          C[cbase + (idx_off(ta.Ci, i) + idx_off(ta.Cj, jr >> 1)) * 2 + (jr & 1)] = (TC)val;
        }
      }
}

// sum the split-K partials in FP64 and scatter to C through its index maps
template <bool CPLX, class TC>
__global__ void k_splitk_reduce(const double* __restrict__ partial, TC* __restrict__ C, GemmNT d, int ksplit) {
  const int Nr = CPLX ? 2 * d.N : d.N;
  const long long per = (long long)d.M * Nr, tot = per * d.batch;
  constexpr int CW = CPLX ? 2 : 1;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int item = (int)(e / per);
    const long long r = e % per;
    const int i = (int)(r / Nr), jr = (int)(r % Nr);
    double s = 0.0;
    for (int k = 0; k < ksplit; ++k) s += partial[((size_t)k * d.batch + item) * per + r];
    const int j = CPLX ? jr >> 1 : jr, part = CPLX ? jr & 1 : 0;
    C[(idx_off(d.Cb, item) + idx_off(d.Ci, i) + idx_off(d.Cj, j)) * CW + part] = (TC)s;
  }
}

template <int PREC, bool CPLX, class TA, class TB, class TC>
static hipError_t run_mixed(const void* A, const void* B, void* C, const GemmNT& d, int ksplit, double* partial,
                            hipStream_t st, const ProfHook& ph, int kind) {
  const int Mr = d.M, Nr = CPLX ? 2 * d.N : d.N, Kr = CPLX ? 2 * d.K : d.K;
  MixedArgs a{};
  a.d = d;
  a.ksplit = ksplit < 1 ? 1 : ksplit;
  int chunk = (Kr + a.ksplit - 1) / a.ksplit;
  chunk = (chunk + MT_BK - 1) / MT_BK * MT_BK;
  a.kchunk = chunk;
  a.ksplit = (Kr + chunk - 1) / chunk;
  a.partial = partial;
  dim3 g((Nr + MT_BN - 1) / MT_BN, (Mr + MT_BM - 1) / MT_BM, d.batch * a.ksplit), b(256);
  ph(kind, 0);
  hipLaunchKernelGGL((k_mfma_nt<PREC, CPLX, TA, TB, TC>), g, b, 0, st, (const TA*)A, (const TB*)B, (TC*)C, a);
  ph(kind, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.ksplit == 1) return e;
  long long tot = (long long)Mr * Nr * d.batch;
  int gx = (int)std::min<long long>((tot + 255) / 256, 4096);
  ph(PK_E6RED, 0);
  hipLaunchKernelGGL((k_splitk_reduce<CPLX, TC>), dim3(gx), dim3(256), 0, st, partial, (TC*)C, d, a.ksplit);
  ph(PK_E6RED, 1);
  return hipGetLastError();
}

// all offsets of an index map even (in scalars)
static bool idx_even(const Idx3& x, int cw) {
  return ((x.s0 * cw) % 2 == 0) && ((x.s1 * cw) % 2 == 0) && ((x.s2 * cw) % 2 == 0);
}

template <int PREC, bool CPLX, class TA, class TB, class TC>
static hipError_t run_tile(const void* A, const void* B, void* C, const GemmNT& d, int ksplit, double* partial,
                           hipStream_t st, const ProfHook& ph, int kind) {
  constexpr int CW = CPLX ? 2 : 1;
  const int Mr = d.M, Nr = CW * d.N, Kr = CW * d.K;
  TileArgs a{};
  a.d = d;
  a.tiles_m = (Mr + TL_M - 1) / TL_M;
  a.tiles_n = (Nr + TL_N - 1) / TL_N;
  a.ksplit = ksplit < 1 ? 1 : ksplit;
  int chunk = (Kr + a.ksplit - 1) / a.ksplit;
  chunk = (chunk + TL_K - 1) / TL_K * TL_K;
  a.kchunk = chunk;
  a.ksplit = (Kr + chunk - 1) / chunk;
  a.nwork = a.tiles_m * a.tiles_n * a.ksplit * d.batch;
  a.partial = partial;
  const bool vec = (Kr % 2 == 0) && idx_even(d.Ab, CW) && idx_even(d.Ai, CW) && idx_even(d.Bb, CW) &&
                   idx_even(d.Bj, CW) && ((uintptr_t)A % (2 * sizeof(TA)) == 0) && ((uintptr_t)B % (2 * sizeof(TB)) == 0);
  const int per = (a.nwork + 7) / 8;
  dim3 g(8 * per), b(TL_THREADS);
  ph(kind, 0);
  if (vec)
    hipLaunchKernelGGL((k_mfma_tile<PREC, CPLX, 2, TA, TB, TC>), g, b, 0, st, (const TA*)A, (const TB*)B, (TC*)C, a);
  else
    hipLaunchKernelGGL((k_mfma_tile<PREC, CPLX, 1, TA, TB, TC>), g, b, 0, st, (const TA*)A, (const TB*)B, (TC*)C, a);
  ph(kind, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.ksplit == 1) return e;
  long long tot = (long long)Mr * Nr * d.batch;
  int gx = (int)std::min<long long>((tot + 255) / 256, 4096);
  ph(PK_E6RED, 0);
  hipLaunchKernelGGL((k_splitk_reduce<CPLX, TC>), dim3(gx), dim3(256), 0, st, partial, (TC*)C, d, a.ksplit);
  ph(PK_E6RED, 1);
  return hipGetLastError();
}

// E6 in FP16X3 from the pre-split rows of the fused kernels (complex):
// A rows (L2) and B rows (Right) of Kc complex entries, 2 Kc words each,
// item strides in words; output through the maps of d (C side only)
template <int WY>
static hipError_t run_tile_f16_w(const void* A, const void* B, void* C, const GemmNT& d, long long a_item,
                                 long long b_item, const float* sA, const float* sB, int ksplit, double* partial,
                                 hipStream_t st, const ProfHook& ph, int kind) {
  const int Mr = d.M, Nr = 2 * d.N, Kr = 2 * d.K;
  TileF16Args a{};
  a.M = d.M; a.N = d.N; a.Kc = d.K; a.batch = d.batch;
  a.a_item = a_item; a.b_item = b_item;
  a.a_row = 2LL * d.K; a.b_row = 2LL * d.K;
  a.sA = sA; a.sB = sB;
  a.Cb = d.Cb; a.Ci = d.Ci; a.Cj = d.Cj;
  a.tiles_m = (Mr + TL_M - 1) / TL_M;
  a.tiles_n = (Nr + 64 * WY - 1) / (64 * WY);
  a.ksplit = ksplit < 1 ? 1 : ksplit;
  int chunk = (Kr + a.ksplit - 1) / a.ksplit;
  chunk = (chunk + TL_K - 1) / TL_K * TL_K;
  a.kchunk = chunk;
  a.ksplit = (Kr + chunk - 1) / chunk;
  a.nwork = a.tiles_m * a.tiles_n * a.ksplit * d.batch;
  a.partial = partial;
  const int per = (a.nwork + 7) / 8;
  ph(kind, 0);
  hipLaunchKernelGGL((k_mfma_tile_f16<double, WY>), dim3(8 * per), dim3(TL_THREADS), 0, st, (const unsigned*)A,
                     (const unsigned*)B, (double*)C, a);
  ph(kind, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.ksplit == 1) return e;
  long long tot = (long long)Mr * Nr * d.batch;
  int gx = (int)std::min<long long>((tot + 255) / 256, 4096);
  ph(PK_E6RED, 0);
  hipLaunchKernelGGL((k_splitk_reduce<true, double>), dim3(gx), dim3(256), 0, st, partial, (double*)C, d, a.ksplit);
  ph(PK_E6RED, 1);
  return hipGetLastError();
}

// the FP16X3 assembly with output tiles of 64 wy columns (wy 2 or 4; any
// other value takes the default F16_WY; the load mapping needs wy >= 2)
static hipError_t run_tile_f16(const void* A, const void* B, void* C, const GemmNT& d, long long a_item,
                               long long b_item, const float* sA, const float* sB, int ksplit, double* partial,
                               hipStream_t st, const ProfHook& ph, int kind, int wy) {
  switch (wy) {
    case 4: return run_tile_f16_w<4>(A, B, C, d, a_item, b_item, sA, sB, ksplit, partial, st, ph, kind);
    default: return run_tile_f16_w<F16_WY>(A, B, C, d, a_item, b_item, sA, sB, ksplit, partial, st, ph, kind);
  }
}

// K chunks of the tiled assembly: about three blocks per CU (one runs at a
// time per CU, so the last round is at most a third of the work), chunks of
// at least 8 steps
static int tile_ksplit(int batch, int M, int Nr, int Kr) {
  const long long tiles = (long long)((M + TL_M - 1) / TL_M) * ((Nr + TL_N - 1) / TL_N) * batch;
  int ks = (int)std::max<long long>(1, (768 + tiles / 2) / std::max<long long>(1, tiles));
  const int kmax = std::max(1, Kr / (8 * TL_K));
  return std::min(ks, std::min(kmax, 32));
}

// number of K chunks for the final assembly: aim at ~2 waves of workgroups on 256 CUs
static int e6_ksplit(int batch, int M, int Nr, int Kr) {
  long long tiles = (long long)((M + MT_BM - 1) / MT_BM) * ((Nr + MT_BN - 1) / MT_BN) * batch;
  int ks = (int)std::max<long long>(1, 512 / std::max<long long>(1, tiles));
  int kmax = std::max(1, Kr / (4 * MT_BK));
  return std::min(ks, std::min(kmax, 16));
}

// largest K split of the final assembly: the heuristic's, or a tuned one of
// at most E6_KS_TUNE_MAX (never more chunks than steps of 8 K tiles allow)
static int e6_ks_cap(bool cplx, int batch, int R, int D) {
  const int M = R * R, Nr = (cplx ? 2 : 1) * R * R, Kr = (cplx ? 2 : 1) * D * D * D * D;
  const int kmax = std::max(1, Kr / (8 * TL_K));
  return std::max(tile_ksplit(batch, M, Nr, Kr), std::min(E6_KS_TUNE_MAX, kmax));
}

size_t mixed_partial_bytes(bool cplx, int batch, int R, int D) {
  const int ks = e6_ks_cap(cplx, batch, R, D);
  return ks > 1 ? (size_t)ks * batch * R * R * (cplx ? 2 : 1) * R * R * sizeof(double) : 0;
}

int e6_ksplit_default(bool cplx, int batch, int R, int D) {
  const int M = R * R, Nr = (cplx ? 2 : 1) * R * R, Kr = (cplx ? 2 : 1) * D * D * D * D;
  return tile_ksplit(batch, M, Nr, Kr);
}

int e6_ksplit_max(bool cplx, int batch, int R, int D) { return e6_ks_cap(cplx, batch, R, D); }

template <int PREC, bool CPLX>
static hipError_t env_heavy(int batch, int p, int D, int R, const void* QXe, const void* QXp, const void* QYe,
                            const void* QYp, const void* ETT, const void* EBT, long long es, long long qs, long long hs,
                            void* H0, void* H1, void* H2, void* g, hipStream_t st, const ProfHook& ph, int e6_ks) {
  using T64 = double;  // scalar of the compute-type inputs
  const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D2 * D2, RD4 = (long long)R * D4;
  const int pD = p * D;
  hipError_t e;
  if (CPLX && e45_supported(CPLX, PREC, D)) {
    // Right, and Left -> L1 -> L2 per (a, a') block, on the matrix cores
    e = launch_env_fused(PREC, batch, p, D, R, QXe, QXp, QYe, QYp, ETT, EBT, es, qs, H0, H1, H2, hs, st, ph);
    if (e != hipSuccess) return e;
  } else {
    // Left / Right
    GemmNT d{};
    d.M = (int)(R * D2); d.N = (int)(R * D2); d.K = pD; d.batch = batch;
    d.Ab = idx1(qs); d.Bb = idx1(qs); d.Cb = idx1(hs);
    d.Ai = idx1(pD); d.Ak = idx1(1); d.Bj = idx1(pD); d.Bk = idx1(1);
    d.conjB = 1;
    d.Ci = idx3(D, D, RD4, D3, D); d.Cj = idx3(D, D, D4, D2, 1);
    e = run_tile<PREC, CPLX, T64, T64, float>(QXe, QXp, H0, d, 1, nullptr, st, ph, PK_LEFTRIGHT);
    if (e != hipSuccess) return e;
    d.Ci = idx3(D, D, RD4, D, D3); d.Cj = idx3(D, D, D4, 1, D2);
    e = run_tile<PREC, CPLX, T64, T64, float>(QYe, QYp, H2, d, 1, nullptr, st, ph, PK_LEFTRIGHT);
    if (e != hipSuccess) return e;
    // L1 = Left x Etop, L2 = L1 x Ebot
    GemmNT f{};
    f.M = (int)(R * R * D2); f.N = (int)D2; f.K = (int)D2; f.batch = batch;
    f.Ab = idx1(hs); f.Bb = idx1(es); f.Cb = idx1(hs);
    f.Ai = idx1(D2); f.Ak = idx1(1); f.Bj = idx1(D2); f.Bk = idx1(1);
    f.Ci = idx2((int)D2, D4, 1); f.Cj = idx1(D2);
    e = run_tile<PREC, CPLX, float, T64, float>(H0, ETT, H1, f, 1, nullptr, st, ph, PK_E4);
    if (e != hipSuccess) return e;
    f.Ci = idx1(D2); f.Cj = idx1(1);
    e = run_tile<PREC, CPLX, float, T64, float>(H1, EBT, H0, f, 1, nullptr, st, ph, PK_E5);
    if (e != hipSuccess) return e;
  }
  // g = L2 Right^T with split K, FP64 reduction
  GemmNT q{};
  q.M = R * R; q.N = R * R; q.K = (int)D4; q.batch = batch;
  q.Ab = idx1(hs); q.Bb = idx1(hs); q.Cb = idx1((long long)R * R * R * R);
  q.Ai = idx1(D4); q.Ak = idx1(1); q.Bj = idx1(D4); q.Bk = idx1(1);
  q.Ci = idx2(R, R, (long long)R * R * R); q.Cj = idx2(R, 1, (long long)R * R);
  const int Nr = (CPLX ? 2 : 1) * q.N, Kr = (CPLX ? 2 : 1) * q.K;
  // the tuned schedule when one is given: K split in the low byte (at most
  // the reserved e6_ks_cap), FP16X3 tile width code above it
  const int ksq = e6_ks & 0xff, wy = (e6_ks >> 8) & 0xff;
  const int ks = ksq > 0 ? std::min(ksq, e6_ks_cap(CPLX, batch, R, D)) : tile_ksplit(batch, q.M, Nr, Kr);
  // partial sums live right after H2 (the workspace reserves mixed_partial_bytes there)
  double* partial = (double*)((char*)H2 + (size_t)batch * hs * (CPLX ? 8 : 4));
  if constexpr (PREC == NTU_PREC_FP16X3 && CPLX) {
    // the fused kernels wrote L2 and Right as scaled float16 pieces
    const E45Scales sc = e45_scales(H1, PREC, batch, D, R);
    return run_tile_f16(H0, H2, g, q, 2 * hs, 2 * hs, sc.left, sc.right, ks, partial, st, ph, PK_E6, wy);
  }
  return run_tile<PREC, CPLX, float, float, T64>(H0, H2, g, q, ks, partial, st, ph, PK_E6);
}

hipError_t launch_env_heavy_mixed(bool cplx, int precision, int batch, int p, int D, int R, const void* QXe,
                                  const void* QXp, const void* QYe, const void* QYp, const void* ETT,
                                  const void* EBT, long long es, long long qs, long long hs, void* H0, void* H1,
                                  void* H2, void* g, hipStream_t st, const ProfHook& ph, int e6_ks) {
#define NTU_MIX(P, C) return env_heavy<P, C>(batch, p, D, R, QXe, QXp, QYe, QYp, ETT, EBT, es, qs, hs, H0, H1, H2, g, st, ph, e6_ks)
  if (precision == NTU_PREC_BF16X3) { if (cplx) NTU_MIX(NTU_PREC_BF16X3, true); NTU_MIX(NTU_PREC_BF16X3, false); }
  if (precision == NTU_PREC_BF16X6) { if (cplx) NTU_MIX(NTU_PREC_BF16X6, true); NTU_MIX(NTU_PREC_BF16X6, false); }
  // FP16X3: the fused path only (complex, D^2 <= 64), where the operands are
  // scaled block by block and E6 takes them pre-split
  if (precision == NTU_PREC_FP16X3 && cplx && e45_supported(cplx, precision, D)) NTU_MIX(NTU_PREC_FP16X3, true);
  return hipErrorNotSupported;
#undef NTU_MIX
}

}  // namespace ntu
