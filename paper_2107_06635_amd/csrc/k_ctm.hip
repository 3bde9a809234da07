// Device primitives of the CTMRG expectation values: permutation of tensor
// axes, complex products, normalisation by the largest modulus, and the
// leading left singular vectors of a matrix (the isometry of a cut).
#include "ctm.h"
#include "linalg.h"

namespace ntu {

struct PermArgs {
  int rank;
  int out_shape[CTM_MAX_RANK];
  long long in_stride[CTM_MAX_RANK];  // stride in the input of out's axis k
};

__global__ void __launch_bounds__(256) k_ctm_permute(const cd* __restrict__ in, cd* __restrict__ out, long long n,
                                                     PermArgs a, int conj) {
  for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < n; o += (long long)gridDim.x * blockDim.x) {
    long long rem = o, src = 0;
    for (int k = a.rank - 1; k >= 0; --k) {
      const long long i = rem % a.out_shape[k];
      rem /= a.out_shape[k];
      src += i * a.in_stride[k];
    }
    const cd v = in[src];
    out[o] = conj ? conjv(v) : v;
  }
}

static int grid_for(long long n, int bs) {
  long long g = (n + bs - 1) / bs;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

hipError_t ctm_permute(const cd* in, cd* out, int rank, const int* in_shape, const int* perm, bool conj,
                       hipStream_t st) {
  if (rank < 1 || rank > CTM_MAX_RANK) return hipErrorInvalidValue;
  long long stride[CTM_MAX_RANK];
  long long s = 1, n = 1;
  for (int k = rank - 1; k >= 0; --k) {
    stride[k] = s;
    s *= in_shape[k];
  }
  PermArgs a{};
  a.rank = rank;
  for (int k = 0; k < rank; ++k) {
    a.out_shape[k] = in_shape[perm[k]];
    a.in_stride[k] = stride[perm[k]];
    n *= a.out_shape[k];
  }
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctm_permute, dim3(grid_for(n, 256)), dim3(256), 0, st, in, out, n, a, conj ? 1 : 0);
  return hipGetLastError();
}

// 32 x 32 tile of C per workgroup of 256 threads (2 x 2 outputs each), K in
// chunks of 16 through shared memory; out-of-range operands read as zero.
// One 32 x 32 tile of C per workgroup over the K range [z kc, min(K, (z + 1) kc))
// of blockIdx.z = z, written to C + z cstride (z = 0, kc = K: C itself).
__global__ void __launch_bounds__(256) k_ctm_gemm(const cd* __restrict__ A, const cd* __restrict__ B,
                                                  cd* __restrict__ C, int M, int N, int K, int kc,
                                                  long long cstride) {
  constexpr int T = 32, KC = 16;
  __shared__ cd As[KC][T + 1];
  __shared__ cd Bs[KC][T + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * T, j0 = blockIdx.x * T;
  const int kb0 = blockIdx.z * kc, kend = min(K, kb0 + kc);
  C += blockIdx.z * cstride;
  cd acc[2][2] = {{cd{0, 0}, cd{0, 0}}, {cd{0, 0}, cd{0, 0}}};
  for (int k0 = kb0; k0 < kend; k0 += KC) {
    for (int e = tid; e < KC * T; e += 256) {
      const int r = e / KC, kk = e % KC;            // A: row r of the tile, column kk of the chunk
      const int i = i0 + r, k = k0 + kk;
      As[kk][r] = (i < M && k < kend) ? A[(long long)i * K + k] : cd{0, 0};
      const int kb = e / T, c = e % T;              // B: row kb of the chunk, column c of the tile
      const int kk2 = k0 + kb, j = j0 + c;
      Bs[kb][c] = (kk2 < kend && j < N) ? B[(long long)kk2 * N + j] : cd{0, 0};
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const cd a0 = As[kk][ty], a1 = As[kk][ty + 16];
      const cd b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const int i = i0 + ty + 16 * u, j = j0 + tx + 16 * v;
      if (i < M && j < N) C[(long long)i * N + j] = acc[u][v];
    }
}

// C[e] = sum_z P[z mn + e], z = 0 .. S - 1 in order
__global__ void k_ctm_sum_splits(const cd* __restrict__ P, cd* __restrict__ C, long long mn, int S) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < mn; e += (long long)gridDim.x * blockDim.x) {
    cd t{0.0, 0.0};
    for (int z = 0; z < S; ++z) t += P[z * mn + e];
    C[e] = t;
  }
}

hipError_t ctm_gemm(const cd* A, const cd* B, cd* C, int M, int N, int K, cd* ws, long long ws_el, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int tiles = ((N + 31) / 32) * ((M + 31) / 32);
  const long long mn = (long long)M * N;
  // few output tiles over a long K: the K range split over S workgroups per
  // tile (at least 512 columns of K each, about 512 workgroups in all), the
  // partial tiles summed in order by a second launch
  int S = 1;
  if (ws && tiles < 128 && K >= 1024) {
    S = (int)std::min<long long>({(long long)(512 + tiles - 1) / tiles, (long long)K / 512, ws_el / mn, 1024});
    if (S < 2) S = 1;
  }
  if (S == 1) {
    hipLaunchKernelGGL(k_ctm_gemm, dim3((N + 31) / 32, (M + 31) / 32, 1), dim3(256), 0, st, A, B, C, M, N, K, K, 0ll);
    return hipGetLastError();
  }
  const int kc = ((K + S - 1) / S + 15) & ~15;
  S = (K + kc - 1) / kc;  // every split non-empty
  hipLaunchKernelGGL(k_ctm_gemm, dim3((N + 31) / 32, (M + 31) / 32, S), dim3(256), 0, st, A, B, ws, M, N, K, kc, mn);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ctm_sum_splits, dim3(grid_for(mn, 256)), dim3(256), 0, st, ws, C, mn, S);
  return hipGetLastError();
}

// The same tiles with the operands gathered and the result scattered through
// separable offsets: entry (i, k) of A is A[off(ra, i) + off(ca, k)], where
// off(g, x) splits x into the digits of g's axes (last axis fastest) and sums
// digit times stride; likewise B (rows rb, columns cb) and C (rc, cc).
// conj_a, conj_b conjugate the operands on load.
NTU_DEV long long gather_off(const CtmAxes& g, int x) {
  long long o = 0;
  for (int a = g.n - 1; a >= 0; --a) {
    const int q = x / g.dim[a];
    o += (long long)(x - q * g.dim[a]) * g.stride[a];
    x = q;
  }
  return o;
}

__global__ void __launch_bounds__(256) k_ctm_gemm_gather(const cd* __restrict__ A, const cd* __restrict__ B,
                                                         cd* __restrict__ C, int M, int N, int K, CtmGather gd) {
  constexpr int T = 32, KC = 16;
  __shared__ cd As[KC][T + 1];
  __shared__ cd Bs[KC][T + 1];
  __shared__ long long offA[T], offB[T], kA[KC], kB[KC];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * T, j0 = blockIdx.x * T;
  if (tid < T) offA[tid] = i0 + tid < M ? gather_off(gd.ra, i0 + tid) : 0;
  else if (tid < 2 * T) offB[tid - T] = j0 + tid - T < N ? gather_off(gd.cb, j0 + tid - T) : 0;
  cd acc[2][2] = {{cd{0, 0}, cd{0, 0}}, {cd{0, 0}, cd{0, 0}}};
  for (int k0 = 0; k0 < K; k0 += KC) {
    if (tid < KC) kA[tid] = k0 + tid < K ? gather_off(gd.ca, k0 + tid) : 0;
    else if (tid < 2 * KC) kB[tid - KC] = k0 + tid - KC < K ? gather_off(gd.rb, k0 + tid - KC) : 0;
    __syncthreads();
    for (int e = tid; e < KC * T; e += 256) {
      const int r = e / KC, kk = e % KC;
      const int i = i0 + r, k = k0 + kk;
      cd a = (i < M && k < K) ? A[offA[r] + kA[kk]] : cd{0, 0};
      if (gd.conj_a) a.y = -a.y;
      As[kk][r] = a;
      const int kb = e / T, c = e % T;
      const int kk2 = k0 + kb, j = j0 + c;
      cd b = (kk2 < K && j < N) ? B[kB[kb] + offB[c]] : cd{0, 0};
      if (gd.conj_b) b.y = -b.y;
      Bs[kb][c] = b;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const cd a0 = As[kk][ty], a1 = As[kk][ty + 16];
      const cd b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const int i = i0 + ty + 16 * u, j = j0 + tx + 16 * v;
      if (i < M && j < N) C[gather_off(gd.rc, i) + gather_off(gd.cc, j)] = acc[u][v];
    }
}

hipError_t ctm_gemm_gather(const cd* A, const cd* B, cd* C, int M, int N, int K, const CtmGather& gd,
                           hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  for (const CtmAxes* g : {&gd.ra, &gd.ca, &gd.rb, &gd.cb, &gd.rc, &gd.cc})
    if (g->n < 0 || g->n > CTM_MAX_RANK) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ctm_gemm_gather, dim3((N + 31) / 32, (M + 31) / 32), dim3(256), 0, st, A, B, C, M, N, K, gd);
  return hipGetLastError();
}

__global__ void k_ctm_widen(const double* __restrict__ src, cd* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = cd{src[i], 0.0};
}

hipError_t ctm_widen(const double* src, cd* dst, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctm_widen, dim3(grid_for(n, 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

__global__ void k_ctm_zero(cd* x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = cd{0.0, 0.0};
}

hipError_t ctm_zero(cd* x, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctm_zero, dim3(grid_for(n, 256)), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

// Largest modulus: non-negative doubles order like their bit patterns, so an
// unsigned 64-bit atomic maximum on the pattern gives the maximum.
__global__ void k_ctm_clear_slot(unsigned long long* slot) { *slot = 0ull; }
__global__ void __launch_bounds__(256) k_ctm_maxabs(const cd* __restrict__ x, long long n, unsigned long long* slot) {
  double m = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    m = fmax(m, absv(x[i]));
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) atomicMax(slot, (unsigned long long)__double_as_longlong(m));
}
__global__ void k_ctm_scale(cd* x, long long n, const unsigned long long* slot) {
  const double m = __longlong_as_double((long long)*slot);
  if (!(m > 0.0)) return;
  const double inv = 1.0 / m;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = x[i] * inv;
}

hipError_t ctm_normalise(cd* x, long long n, unsigned long long* slot, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctm_clear_slot, dim3(1), dim3(1), 0, st, slot);
  const int g = grid_for(n, 256);
  hipLaunchKernelGGL(k_ctm_maxabs, dim3(g), dim3(256), 0, st, x, n, slot);
  hipLaunchKernelGGL(k_ctm_scale, dim3(g), dim3(256), 0, st, x, n, (const unsigned long long*)slot);
  return hipGetLastError();
}

// Leading left singular vectors of an n x n matrix rho by one-sided
// (Hestenes) Jacobi: the columns of W = rho are rotated pairwise, W <- W J
// with J the 2 x 2 unitary that makes the pair orthogonal, until every pair
// is; then W = U Sigma, and the k columns of largest norm, normalised, are
// u_1..u_k.  The singular values are not squared, so a column of norm
// sigma_j keeps its direction to about eps sigma_1 / sigma_j, which the
// network weighs by sigma_j.  A pair is left alone when its inner product is
// below tol sqrt(|w_p|^2 |w_q|^2), tol = 4 eps sqrt(n) (the rounding floor
// of an n-term inner product, so a sweep with no rotation does come), or
// below (1e-15 ||rho||_F)^2.  Gram-Schmidt twice over the chosen columns,
// with unit vectors taking the place of columns beyond the numerical rank
// (norm at most CTM_RANK_EPS sigma_1), makes Z orthonormal.

constexpr int SVD_SWEEPS = 40;

// the unitary of one pair from its Gram entries al = |w_p|^2, be = |w_q|^2,
// ga = w_p^H w_q: with y = e^{-i arg ga} w_q the pair becomes real, and the
// plane rotation (c, s) with t = s / c the smaller root of
// t^2 + 2 zeta t - 1 = 0, zeta = (be - al) / (2 |ga|), zeroes its inner
// product: w_p <- c w_p - s y, w_q <- s w_p + c y.  False: nothing to do.
NTU_DEV bool hestenes_params(double al, double be, cd ga, double tiny, double tol, double& c, double& s, cd& em,
                             double& tg) {
  // the tests on squares (g^2 against tiny^2 and tol^2 al be): one square
  // root fewer per pair; the values here are far from the overflow range
  const double g2 = abs2(ga);
  if (!(g2 > tiny * tiny) || !(g2 > tol * tol * al * be)) return false;
  // 1 / |ga| and c = 1 / sqrt(1 + t^2) as reciprocal square roots (one
  // dependent operation each instead of a square root and a division)
  const double ig = rsqrt(g2), g = g2 * ig;
  const double zeta = 0.5 * (be - al) * ig;
  const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  c = rsqrt(1.0 + t * t);
  s = c * t;
  em = cd{ga.x * ig, -ga.y * ig};
  tg = t * g;  // |w_p|^2 falls and |w_q|^2 rises by t |ga|
  return true;
}

template <int PER> NTU_DEV void pair_rotate(cd (&a)[PER], cd (&b)[PER], double c, double s, cd em) {
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const cd y = em * b[u];
    const cd an = c * a[u] - s * y;
    b[u] = s * a[u] + c * y;
    a[u] = an;
  }
}

// Gram-Schmidt twice over the k columns of Z (n x k, row-major), in order,
// replacing a column with nothing left by the next unit vector; then
// normalised.  Every thread of the workgroup takes part.
NTU_DEV void svd_orthonormalise(cd* Z, int n, int k, double* red, int* pick_sh) {
  const int tid = threadIdx.x;
  int next_unit = 0;
  for (int col = 0; col < k; ++col) {
    for (int attempt = 0; attempt <= n; ++attempt) {
      for (int pass = 0; pass < 2; ++pass)
        for (int b = 0; b < col; ++b) {
          cd dot{0.0, 0.0};
          for (int i = tid; i < n; i += blockDim.x) dot += cmul(Z[(long long)i * k + b], Z[(long long)i * k + col]);
          dot.x = block_sum(dot.x, red);
          dot.y = block_sum(dot.y, red);
          for (int i = tid; i < n; i += blockDim.x)
            Z[(long long)i * k + col] = Z[(long long)i * k + col] - dot * Z[(long long)i * k + b];
          __syncthreads();
        }
      double nn = 0.0;
      for (int i = tid; i < n; i += blockDim.x) nn += abs2(Z[(long long)i * k + col]);
      nn = sqrt(block_sum(nn, red));
      if (nn > 0.5) {
        const double inv = 1.0 / nn;
        for (int i = tid; i < n; i += blockDim.x) Z[(long long)i * k + col] = Z[(long long)i * k + col] * inv;
        __syncthreads();
        break;
      }
      if (tid == 0) *pick_sh = next_unit;
      __syncthreads();
      const int u = *pick_sh;
      for (int i = tid; i < n; i += blockDim.x) Z[(long long)i * k + col] = cd{i == u ? 1.0 : 0.0, 0.0};
      ++next_unit;
      __syncthreads();
    }
  }
}

// The same Gram-Schmidt by one wave: entry (i, c) of Z at zs + i srow +
// c scol (LDS or global memory; n <= 64 PER); no barriers, the column being
// orthogonalised kept in registers.
template <int PER>
NTU_DEV void svd_orthonormalise_wave(cd* zs, long long srow, long long scol, int n, int k) {
  const int lane = threadIdx.x & 63;
  auto at = [&](int i, int c) -> cd& { return zs[(long long)i * srow + (long long)c * scol]; };
  int next_unit = 0;
  for (int col = 0; col < k; ++col) {
    cd zc[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) zc[u] = lane + 64 * u < n ? at(lane + 64 * u, col) : cd{0.0, 0.0};
    for (int attempt = 0; attempt <= n; ++attempt) {
      for (int pass = 0; pass < 2; ++pass)
        for (int b = 0; b < col; ++b) {
          cd dot{0.0, 0.0};
#pragma unroll
          for (int u = 0; u < PER; ++u)
            if (lane + 64 * u < n) dot += cmul(at(lane + 64 * u, b), zc[u]);
          dot = wave_sum(dot);
#pragma unroll
          for (int u = 0; u < PER; ++u)
            if (lane + 64 * u < n) zc[u] = zc[u] - dot * at(lane + 64 * u, b);
        }
      double nn = 0.0;
#pragma unroll
      for (int u = 0; u < PER; ++u) nn += abs2(zc[u]);
      nn = sqrt(wave_sum(nn));
      if (nn > 0.5) {
        const double inv = 1.0 / nn;
#pragma unroll
        for (int u = 0; u < PER; ++u) zc[u] = zc[u] * inv;
        break;
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) zc[u] = cd{lane + 64 * u == next_unit ? 1.0 : 0.0, 0.0};
      ++next_unit;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (lane + 64 * u < n) at(lane + 64 * u, col) = zc[u];
  }
}

// rank_of[j] = the place of column j when the norms nrm[0..n) are sorted
// descending (ties by index).  Returns the floor below which a column counts
// as beyond the numerical rank: CTM_RANK_EPS times the largest norm.  Such
// columns are written as zeros, so that the Gram-Schmidt completion puts
// unit vectors in their place: any orthonormal completion is a singular
// basis there, and this one is reproducible.
NTU_DEV double svd_rank(const double* nrm, int* rank_of, int n) {
  double mx = 0.0;
  for (int j = 0; j < n; ++j) mx = fmax(mx, nrm[j]);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int rk = 0;
    for (int j = 0; j < n; ++j) rk += (nrm[j] > nrm[i] || (nrm[j] == nrm[i] && j < i)) ? 1 : 0;
    rank_of[i] = rk;
  }
  __syncthreads();
  return CTM_RANK_EPS * mx;
}

// y[first..C) moved one place down, y[first] to the end (with the squared
// norms ny kept beside them)
template <int PER, int C, int FIRST> NTU_DEV void shift_cols(cd (&y)[C][PER], double (&ny)[C]) {
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const cd t = y[FIRST][u];
#pragma unroll
    for (int c = FIRST; c < C - 1; ++c) y[c][u] = y[c + 1][u];
    y[C - 1][u] = t;
  }
  const double t = ny[FIRST];
#pragma unroll
  for (int c = FIRST; c < C - 1; ++c) ny[c] = ny[c + 1];
  ny[C - 1] = t;
}

// NP disjoint pairs (a[ia + i], b[ib + di i]), i < NP: inner products summed
// over the wave side by side, then rotated, the squared norms na, nb moved
// along; returns the rotations made
template <int PER, int C, int NP>
NTU_DEV int svd_pairs(cd (&a)[C][PER], cd (&b)[C][PER], double (&na)[C], double (&nb)[C], int ia, int ib, int di,
                      double tiny, double tol) {
  cd ga[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    ga[i] = cd{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < PER; ++u) ga[i] += cmul(a[ia + i][u], b[ib + di * i][u]);
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) ga[i] = wave_sum(ga[i]);
  int rot = 0;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double cs, sn, tg;
    cd em;
    if (hestenes_params(na[ia + i], nb[ib + di * i], ga[i], tiny, tol, cs, sn, em, tg)) {
      pair_rotate<PER>(a[ia + i], b[ib + di * i], cs, sn, em);
      na[ia + i] = fmax(na[ia + i] - tg, 0.0);  // recomputed exactly each round
      nb[ib + di * i] += tg;
      ++rot;
    }
  }
  return rot;
}

// squared norms of the columns a wave holds (exact, once a round)
template <int PER, int C> NTU_DEV void col_norms(const cd (&y)[C][PER], double (&ny)[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) v += abs2(y[c][u]);
    ny[c] = v;
  }
#pragma unroll
  for (int c = 0; c < C; ++c) ny[c] = wave_sum(ny[c]);
}

struct SvdBatch {
  const cd* rho[CTM_SVD_BATCH];
  cd* Z[CTM_SVD_BATCH];
  cd* W[CTM_SVD_BATCH];
};

// n <= 64 * PER and n <= 32 * C: the columns live in registers, in blocks of
// C; wave w holds two blocks (rows lane + 64 u, u < PER), pairs its own
// columns and passes the blocks on through LDS in round-robin order of the
// blocks, so that every two columns meet once a sweep (the pairs inside a
// block at the sweep's first round).  Dynamic LDS: (number of blocks) * C *
// 64 entries.
template <int PER, int C, int ILP, int NT>
__global__ void __launch_bounds__(NT) k_ctm_svd_reg(SvdBatch bt, int n, int k, int zs_cap) {
  extern __shared__ cd xbuf[];
  __shared__ double red[64];
  __shared__ double nrm[CTM_SVD_REG_NMAX];
  __shared__ int rank_of[CTM_SVD_REG_NMAX];
  __shared__ cd rowbuf[2 * 64 * PER];
  __shared__ int cnt, pick_sh;
  const cd* __restrict__ rho = bt.rho[blockIdx.x];
  cd* __restrict__ Z = bt.Z[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = (n + C - 1) / C, nb = nblk + (nblk & 1), nw = nb / 2;
  const bool active = wave < nw;
  const int me = active ? wave : 0;
  cd x[2][C][PER];
  int blk[2];
  rr_pair(nb, 0, me, blk[0], blk[1]);
  double fro = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int col = blk[h] * C + c, row = lane + 64 * u;
        const cd v = active && col < n && row < n ? rho[(long long)row * n + col] : cd{0.0, 0.0};
        x[h][c][u] = v;
        fro += abs2(v);
      }
  fro = block_sum(fro, red);
  // rho = L Q by Householder reflections from the right: row j of what is
  // left, (r_j, .., r_{n-1}), becomes L[j, j] e_j with
  // H = I - beta u u^H, u = conj(r) + conj(e) |r| e_j, e = r_j / |r_j|,
  // beta = 1 / (|r| (|r| + |r_j|)), L[j, j] = -e |r|.  The rows of L are
  // graded where rho's singular values spread over many orders, and the
  // Jacobi sweeps on L's columns (left singular vectors those of rho) then
  // end in a few rounds instead of tens.  Row sums of the update through
  // LDS, one partial per wave.
  for (int j = 0; j < n; ++j) {
    // row j, double-buffered by step so that a wave still updating with
    // step j's row never sees step j + 1's
    cd* const rb = rowbuf + (j & 1) * 64 * PER;
    if (active && lane == (j & 63))
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int label = blk[h] * C + c;
          if (label >= j && label < n) {
            cd v{0.0, 0.0};
#pragma unroll
            for (int u = 0; u < PER; ++u)
              if (u == (j >> 6)) v = x[h][c][u];
            rb[label] = v;
          }
        }
    __syncthreads();
    double s2 = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int col = lane + 64 * u;
      if (col >= j && col < n) s2 += abs2(rb[col]);
    }
    const double nr = sqrt(wave_sum(s2));
    if (!(nr > 0.0)) continue;  // row already zero beyond the diagonal
    const cd rj = rb[j];
    const double arj = absv(rj);
    const cd e = arj > 0.0 ? cd{rj.x / arj, rj.y / arj} : cd{1.0, 0.0};
    const double beta = 1.0 / (nr * (nr + arj));
    const cd uj = conjv(e) * (arj + nr);
    // u_c: column c's entry of the reflector (conj of the row beyond j)
    auto ucol = [&](int label) -> cd {
      return label == j ? uj : (label > j && label < n ? conjv(rb[label]) : cd{0.0, 0.0});
    };
    cd wp[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) wp[u] = cd{0.0, 0.0};
    if (active)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const cd uv = ucol(blk[h] * C + c);
#pragma unroll
          for (int u = 0; u < PER; ++u) wp[u] += x[h][c][u] * uv;
        }
    if (active)
#pragma unroll
      for (int u = 0; u < PER; ++u) xbuf[wave * 64 * PER + lane + 64 * u] = wp[u];
    __syncthreads();
    if (active) {
      cd w[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        w[u] = cd{0.0, 0.0};
        for (int v = 0; v < nw; ++v) w[u] += xbuf[v * 64 * PER + lane + 64 * u];
        w[u] = w[u] * beta;
      }
      const cd ljj = cd{-e.x * nr, -e.y * nr};
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int label = blk[h] * C + c;
          if (label >= j && label < n) {
            const cd ucc = conjv(ucol(label));
#pragma unroll
            for (int u = 0; u < PER; ++u) {
              const int row = lane + 64 * u;
              if (row == j)
                x[h][c][u] = label == j ? ljj : cd{0.0, 0.0};
              else
                x[h][c][u] = x[h][c][u] - w[u] * ucc;
            }
          }
        }
    }
    // the partial sums are next written after the next step's barrier, which
    // every wave reaches only once it has read them
  }
  const double tiny = 1e-30 * fro, tol = 4.0 * 2.220446049250313e-16 * sqrt((double)n);
  for (int sweep = 0; sweep < SVD_SWEEPS; ++sweep) {
    if (tid == 0) cnt = 0;
    __syncthreads();
    int rot = 0;
    for (int r = 0; r < nb - 1; ++r) {
      if (active) {
        double nq[2][C];
        col_norms<PER, C>(x[0], nq[0]);
        col_norms<PER, C>(x[1], nq[1]);
        if (r == 0) {
          // pairs inside each block (circle method on its C columns: the
          // first stays, the others move one place a round)
#pragma unroll 1
          for (int t = 0; t < C - 1; ++t) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
              rot += svd_pairs<PER, C, C / 2>(x[h], x[h], nq[h], nq[h], 0, C - 1, -1, tiny, tol);
            shift_cols<PER, C, 1>(x[0], nq[0]);
            shift_cols<PER, C, 1>(x[1], nq[1]);
          }
        }
        // pairs across the two blocks: column i of one with column i of the
        // other, the second block moving one place a shift
#pragma unroll 1
        for (int sh = 0; sh < C; ++sh) {
#pragma unroll
          for (int i0 = 0; i0 < C; i0 += ILP)
            rot += svd_pairs<PER, C, ILP>(x[0], x[1], nq[0], nq[1], i0, i0, 1, tiny, tol);
          shift_cols<PER, C, 0>(x[1], nq[1]);
        }
      }
      // hand the blocks on to the next round's holders
      int nxt[2];
      rr_pair(nb, r + 1 < nb - 1 ? r + 1 : 0, me, nxt[0], nxt[1]);
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        if (active)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < C; ++c) xbuf[(blk[h] * C + c) * 64 + lane] = x[h][c][u];
        __syncthreads();
        if (active)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < C; ++c) x[h][c][u] = xbuf[(nxt[h] * C + c) * 64 + lane];
        __syncthreads();
      }
      blk[0] = nxt[0];
      blk[1] = nxt[1];
    }
    if (rot && lane == 0) atomicAdd(&cnt, rot);
    __syncthreads();
    const int done = cnt == 0;
    __syncthreads();
    if (done) break;
  }
  // column norms, their order, the k largest columns normalised into Z
  for (int j = tid; j < nb * C; j += blockDim.x) nrm[j] = 0.0;
  __syncthreads();
  if (active)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < PER; ++u) v += abs2(x[h][c][u]);
        v = wave_sum(v);
        if (lane == 0) nrm[blk[h] * C + c] = sqrt(v);
      }
  __syncthreads();
  const double floor_nrm = svd_rank(nrm, rank_of, n);
  // Z staged in LDS when it fits (column c at zs + c * 64 PER), else in
  // global memory
  constexpr int LD = 64 * PER;
  const bool in_lds = k * LD <= zs_cap;
  if (active)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int col = blk[h] * C + c;
        if (col < n && rank_of[col] < k) {
          const double nv = nrm[col];
          const double inv = nv > floor_nrm ? 1.0 / nv : 0.0;
          const int rk = rank_of[col];
#pragma unroll
          for (int u = 0; u < PER; ++u) {
            const int row = lane + 64 * u;
            if (in_lds)
              xbuf[rk * LD + row] = x[h][c][u] * inv;
            else if (row < n)
              Z[(long long)row * k + rk] = x[h][c][u] * inv;
          }
        }
      }
  __syncthreads();
  if (in_lds) {
    if (wave == 0) svd_orthonormalise_wave<PER>(xbuf, 1, LD, n, k);
    __syncthreads();
    for (int e = tid; e < n * k; e += blockDim.x) {
      const int i = e / k, c = e % k;
      Z[(long long)i * k + c] = xbuf[c * LD + i];
    }
  } else {
    svd_orthonormalise(Z, n, k, red, &pick_sh);
  }
}

// n > CTM_SVD_REG_NMAX: three kinds of launches on the columns of W in
// global memory (scratch ws[b]: W, n^2 entries with column j contiguous,
// then the rotation counts of the sweeps and ||rho||_F^2):
//   k_ctm_svd_lq     one workgroup per matrix: W = rho, then the LQ
//                    factorisation of k_ctm_svd_reg (the columns of L);
//   k_ctm_svd_round  one round of the round-robin order on blocks of
//                    SVD_MB columns, one workgroup per pair of blocks (all
//                    pairs across them, and at the sweep's first round the
//                    pairs inside them), one wave per column pair at a time;
//                    a sweep's rounds return at once when the sweep before
//                    made no rotation;
//   k_ctm_svd_final  one workgroup per matrix: norms, order, Z, and the
//                    Gram-Schmidt of one wave.
constexpr int SVD_MB = 8;                  // columns per block (one wave each)
constexpr int SVD_SWEEPS_MULTI = SVD_SWEEPS;  // at most this many sweeps (as the register kernel)
constexpr int SVD_SWEEPS_FIRST = 8;        // sweeps launched before the first look at the counts

struct SvdMemWs {
  cd* W;
  int* rot;      // rotations made in each sweep
  double* fro;   // ||rho||_F^2
};
NTU_DEV SvdMemWs svd_mem_ws(cd* base, int n) {
  SvdMemWs w;
  w.W = base;
  w.rot = (int*)(base + (long long)n * n);
  w.fro = (double*)(w.rot + 2 * SVD_SWEEPS_MULTI);
  return w;
}

// The LQ factorisation of k_ctm_svd_reg by panels of bp = min(LQ_BP,
// LQ_PANEL_ENT / n) rows: a panel's rows (their columns j0..n-1) are
// factored in LDS one reflector H_k = 1 - beta_k v_k v_k^H at a time, and
// the rows below take the whole panel at once through the compact form
// H_0 .. H_{b-1} = 1 - V T V^H (T upper triangular, T_kk = beta_k,
// T_ik = -beta_k sum_l T_il v_l^H v_k): W_rest <- W_rest - (W_rest V) T V^H.
constexpr int LQ_PANEL_ENT = 3072;  // entries of a panel (and of V)
constexpr int LQ_BP = 16;           // rows per panel at most
constexpr int LQ_KK = 6;            // sums of Y = W_rest V per thread and pass

__global__ void __launch_bounds__(1024) k_ctm_svd_lq(SvdBatch bt, int n) {
  __shared__ double red[64];
  __shared__ cd Pn[LQ_PANEL_ENT];   // panel row k, column j0 + c at k m + c; then Y at r b + k
  __shared__ cd Vs[LQ_PANEL_ENT];   // v_k at k m + c (zero for c < k)
  __shared__ cd Gm[LQ_BP * LQ_BP];  // v_l^H v_k (l < k) at l LQ_BP + k
  __shared__ cd Tm[LQ_BP * LQ_BP];  // T_ik at i LQ_BP + k (i <= k)
  __shared__ double bet[LQ_BP];
  const cd* __restrict__ rho = bt.rho[blockIdx.x];
  const SvdMemWs ws = svd_mem_ws(bt.W[blockIdx.x], n);
  cd* __restrict__ W = ws.W;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  if (tid < SVD_SWEEPS_MULTI) ws.rot[tid] = 0;
  double fro = 0.0;
  for (long long e = tid; e < (long long)n * n; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const cd v = rho[e];
    W[(long long)j * n + i] = v;
    fro += abs2(v);
  }
  fro = block_sum(fro, red);  // its barriers also publish W
  if (tid == 0) *ws.fro = fro;
  const int bp = min(LQ_BP, LQ_PANEL_ENT / n);
  for (int j0 = 0; j0 < n; j0 += bp) {
    const int b = min(bp, n - j0), m = n - j0;
    for (int e = tid; e < b * m; e += blockDim.x) {
      const int k = e % b, c = e / b;
      Pn[k * m + c] = W[(long long)(j0 + c) * n + j0 + k];
    }
    __syncthreads();
    for (int k = 0; k < b; ++k) {
      cd* const row = Pn + k * m;
      double s2 = 0.0;
      for (int c = k + lane; c < m; c += 64) s2 += abs2(row[c]);
      const double nr = sqrt(wave_sum(s2));  // the same on every wave
      const cd rj = row[k];
      const double arj = absv(rj);
      const cd e = arj > 0.0 ? cd{rj.x / arj, rj.y / arj} : cd{1.0, 0.0};
      const bool act = nr > 0.0;  // else H_k = 1 (the row is zero from k on)
      const double beta = act ? 1.0 / (nr * (nr + arj)) : 0.0;
      const cd uj = conjv(e) * (arj + nr);
      auto ucol = [&](int c) -> cd { return c == k ? uj : conjv(row[c]); };  // c >= k
      for (int c = tid; c < m; c += blockDim.x) Vs[k * m + c] = (c < k || !act) ? cd{0.0, 0.0} : ucol(c);
      if (tid == 0) bet[k] = beta;
      if (act)
        for (int r = k + 1 + wave; r < b; r += nwave) {  // the panel's later rows, a wave each
          cd* const pr = Pn + r * m;
          cd w{0.0, 0.0};
          for (int c = k + lane; c < m; c += 64) w += pr[c] * ucol(c);
          w = wave_sum(w) * beta;
          for (int c = k + lane; c < m; c += 64) pr[c] = pr[c] - w * conjv(ucol(c));
        }
      __syncthreads();
      // row k of L: -e |r| on the diagonal, zeros beyond (the next step
      // reads only rows k + 1 ..)
      if (act)
        for (int c = k + tid; c < m; c += blockDim.x) row[c] = c == k ? cd{-e.x * nr, -e.y * nr} : cd{0.0, 0.0};
    }
    __syncthreads();
    for (int e = tid; e < b * m; e += blockDim.x) {
      const int k = e % b, c = e / b;
      W[(long long)(j0 + c) * n + j0 + k] = Pn[k * m + c];
    }
    const int R = n - j0 - b;  // rows below the panel
    if (R <= 0) break;
    for (int p = wave; p < b * b; p += nwave) {
      const int l = p / b, k = p % b;
      if (l < k) {
        cd g{0.0, 0.0};
        for (int c = lane; c < m; c += 64) g += cmul(Vs[l * m + c], Vs[k * m + c]);
        g = wave_sum(g);
        if (lane == 0) Gm[l * LQ_BP + k] = g;
      }
    }
    __syncthreads();
    if (tid < b) {  // lane i of wave 0 builds row i of T
      const int i = tid;
      Tm[i * LQ_BP + i] = cd{bet[i], 0.0};
      for (int k = i + 1; k < b; ++k) {
        cd t{0.0, 0.0};
        for (int l = i; l < k; ++l) t += Tm[i * LQ_BP + l] * Gm[l * LQ_BP + k];
        Tm[i * LQ_BP + k] = t * (-bet[k]);
      }
    }
    // Y = W_rest V: thread (r, g) sums row j0 + b + r against v_k for
    // k = g, g + ng, ..
    const int Rp = (R + 63) & ~63, ng = (int)blockDim.x / Rp;  // R < n <= 1024: ng >= 1
    const int r = tid % Rp, g = tid / Rp;
    const bool mine = g < ng && r < R;
    cd* const wr = W + j0 + b + r;  // column j0 + c of the row at wr[(j0 + c) n]
    __syncthreads();  // the panel's rows are back in W: Pn takes Y
    // LQ_KK sums per thread and pass (one pass unless b > LQ_KK ng: with
    // 1024 threads ng >= 5 for n <= 204 and b <= 5 for n > 512, so at most
    // five are needed)
    for (int k0 = g; k0 < b; k0 += LQ_KK * ng) {
      cd acc[LQ_KK];
#pragma unroll
      for (int kk = 0; kk < LQ_KK; ++kk) acc[kk] = cd{0.0, 0.0};
      if (mine)
        for (int c0 = 0; c0 < m; c0 += 4) {  // four loads in flight
          cd w[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] = c0 + q < m ? wr[(long long)(j0 + c0 + q) * n] : cd{0.0, 0.0};
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (c0 + q < m)
#pragma unroll
              for (int kk = 0; kk < LQ_KK; ++kk) {
                const int k = k0 + kk * ng;
                if (k < b) acc[kk] += w[q] * Vs[k * m + c0 + q];
              }
        }
      if (mine)
#pragma unroll
        for (int kk = 0; kk < LQ_KK; ++kk) {
          const int k = k0 + kk * ng;
          if (k < b) Pn[r * b + k] = acc[kk];
        }
    }
    __syncthreads();
    // W_rest <- W_rest - (Y T) V^H, thread (r, g) on the columns c = g, g + ng, ..
    cd yt[LQ_BP];
#pragma unroll
    for (int k = 0; k < LQ_BP; ++k) {
      cd t{0.0, 0.0};
      if (mine && k < b)
        for (int l = 0; l <= k; ++l) t += Pn[r * b + l] * Tm[l * LQ_BP + k];
      yt[k] = t;
    }
    if (mine)
      for (int c0 = g; c0 < m; c0 += 2 * ng) {  // two loads in flight
        cd w[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int c = c0 + q * ng;
          w[q] = c < m ? wr[(long long)(j0 + c) * n] : cd{0.0, 0.0};
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int c = c0 + q * ng;
          if (c < m) {
            cd t{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < LQ_BP; ++k)
              if (k < b) t += yt[k] * conjv(Vs[k * m + c]);
            wr[(long long)(j0 + c) * n] = w[q] - t;
          }
        }
      }
    __syncthreads();  // the next panel reads these rows and rewrites Pn, Vs
  }
}

// one pair of columns by one wave, rows in chunks of 64 (read once for the
// inner products, again for the rotation); returns 1 when it rotated
NTU_DEV int svd_mem_pair(cd* wp, cd* wq, int n, bool valid, double tiny, double tol) {
  const int lane = threadIdx.x & 63;
  if (!valid) return 0;
  double al = 0.0, be = 0.0;
  cd ga{0.0, 0.0};
  for (int i = lane; i < n; i += 64) {
    const cd a = wp[i], b = wq[i];
    al += abs2(a);
    be += abs2(b);
    ga += cmul(a, b);
  }
  al = wave_sum(al);
  be = wave_sum(be);
  ga = wave_sum(ga);
  double cs, sn, tg;
  cd em;
  if (!hestenes_params(al, be, ga, tiny, tol, cs, sn, em, tg)) return 0;
  for (int i = lane; i < n; i += 64) {
    const cd a = wp[i], y = em * wq[i];
    wp[i] = cs * a - sn * y;
    wq[i] = sn * a + cs * y;
  }
  return 1;
}

// IN_LDS: the round's two blocks are copied to LDS first (2 SVD_MB n
// entries of dynamic LDS) and back at the end; otherwise every step reads
// and writes W
constexpr int SVD_LDS_NMAX = 576;  // 2 SVD_MB n entries within 144 KB
template <bool IN_LDS>
__global__ void __launch_bounds__(64 * SVD_MB) k_ctm_svd_round(SvdBatch bt, int n, int nb, int sweep, int r) {
  extern __shared__ cd xbuf[];
  const SvdMemWs ws = svd_mem_ws(bt.W[blockIdx.y], n);
  if (sweep > 0 && ws.rot[sweep - 1] == 0) return;  // converged
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int P, Q;
  rr_pair(nb, r, blockIdx.x, P, Q);
  // column i < 2 SVD_MB of the pair: column i % SVD_MB of block P (i <
  // SVD_MB) or Q; beyond n in the last (or the padding) block
  auto gcol = [&](int i) { return (i < SVD_MB ? P : Q) * SVD_MB + i % SVD_MB; };
  auto col = [&](int i) -> cd* { return IN_LDS ? xbuf + (long long)i * n : ws.W + (long long)gcol(i) * n; };
  if (IN_LDS) {
    for (int e = threadIdx.x; e < 2 * SVD_MB * n; e += blockDim.x) {
      const int i = e / n, row = e % n;
      if (gcol(i) < n) xbuf[e] = ws.W[(long long)gcol(i) * n + row];
    }
    __syncthreads();
  }
  const double fro = *ws.fro;
  const double tiny = 1e-30 * fro, tol = 4.0 * 2.220446049250313e-16 * sqrt((double)n);
  int rot = 0;
  if (r == 0) {
    // pairs inside each block: circle method on its SVD_MB columns (the
    // first fixed), SVD_MB / 2 pairs per block a step, one per wave
    for (int t = 0; t < SVD_MB - 1; ++t) {
      const int h = wave / (SVD_MB / 2), k = wave % (SVD_MB / 2);
      auto pos = [&](int slot) {
        if (slot == 0) return 0;
        const int x = slot - 1 + t;
        return 1 + (x >= SVD_MB - 1 ? x - (SVD_MB - 1) : x);
      };
      const int a = h * SVD_MB + pos(k), b = h * SVD_MB + pos(SVD_MB - 1 - k);
      rot += svd_mem_pair(col(a), col(b), n, gcol(a) < n && gcol(b) < n, tiny, tol);
      __syncthreads();
    }
  }
  // pairs across the blocks: column i of P with column (i + sh) of Q
  for (int sh = 0; sh < SVD_MB; ++sh) {
    const int a = wave, b = SVD_MB + (wave + sh) % SVD_MB;
    rot += svd_mem_pair(col(a), col(b), n, gcol(a) < n && gcol(b) < n, tiny, tol);
    __syncthreads();
  }
  if (IN_LDS)
    for (int e = threadIdx.x; e < 2 * SVD_MB * n; e += blockDim.x) {
      const int i = e / n, row = e % n;
      if (gcol(i) < n) ws.W[(long long)gcol(i) * n + row] = xbuf[e];
    }
  if (rot && lane == 0) atomicAdd(&ws.rot[sweep], rot);
}

// 256 threads: the Gram-Schmidt wave keeps a column of up to 1024 rows in
// registers (a wave per SIMD leaves it room)
__global__ void __launch_bounds__(256) k_ctm_svd_final(SvdBatch bt, int n, int k) {
  __shared__ double nrm[CTM_SVD_NMAX];
  __shared__ int rank_of[CTM_SVD_NMAX];
  cd* __restrict__ Z = bt.Z[blockIdx.x];
  const SvdMemWs ws = svd_mem_ws(bt.W[blockIdx.x], n);
  const cd* __restrict__ W = ws.W;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  for (int j = wave; j < n; j += nwave) {
    double v = 0.0;
    for (int i = lane; i < n; i += 64) v += abs2(W[(long long)j * n + i]);
    v = wave_sum(v);
    if (lane == 0) nrm[j] = sqrt(v);
  }
  __syncthreads();
  const double floor_nrm = svd_rank(nrm, rank_of, n);
  for (long long e = tid; e < (long long)n * n; e += blockDim.x) {
    const int j = (int)(e / n), i = (int)(e % n);
    const int rk = rank_of[j];
    if (rk < k) Z[(long long)i * k + rk] = nrm[j] > floor_nrm ? W[e] * (1.0 / nrm[j]) : cd{0.0, 0.0};
  }
  __syncthreads();
  if (wave == 0) svd_orthonormalise_wave<CTM_SVD_NMAX / 64>(Z, k, 1, n, k);
}

// The dynamic LDS limit of a kernel, set once per device (done[dev]; set
// again every call on devices beyond the table).
constexpr int SVD_ATTR_DEVICES = 64;
static hipError_t set_lds_attr(const void* fn, int bytes, bool* done) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const bool in_table = dev >= 0 && dev < SVD_ATTR_DEVICES;
  if (in_table && done[dev]) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess && in_table) done[dev] = true;
  return e;
}

// one workgroup of NT threads per matrix: n <= 2 C (NT / 64) (two blocks
// of C columns per wave) and n <= 64 PER (PER rows per lane)
template <int PER, int C, int ILP, int NT>
static hipError_t launch_svd_reg(const SvdBatch& bt, int count, int n, int k, hipStream_t st) {
  static_assert(C % 2 == 0 && C % ILP == 0, "block shape");
  constexpr int NW = NT / 64;
  constexpr size_t LDS_CAP = (size_t)(2 * NW * C * 64 > NW * 64 * PER ? 2 * NW * C * 64 : NW * 64 * PER) * sizeof(cd);
  static_assert(LDS_CAP <= 144 * 1024, "LDS");
  if (n > 2 * C * NW || n > 64 * PER) return hipErrorInvalidValue;
  static bool attr[SVD_ATTR_DEVICES] = {};
  const hipError_t ea = set_lds_attr((const void*)k_ctm_svd_reg<PER, C, ILP, NT>, (int)LDS_CAP, attr);
  if (ea != hipSuccess) return ea;
  const int nblk = (n + C - 1) / C, nb = nblk + (nblk & 1);
  const size_t ex = (size_t)nb * C * 64, part = (size_t)NW * 64 * PER, zs = (size_t)k * 64 * PER;
  const size_t cap = LDS_CAP / sizeof(cd);
  size_t ent = ex > part ? ex : part;
  if (zs <= cap && zs > ent) ent = zs;  // Z staged in LDS when it fits
  hipLaunchKernelGGL((k_ctm_svd_reg<PER, C, ILP, NT>), dim3(count), dim3(NT), ent * sizeof(cd), st, bt, n, k,
                     (int)ent);
  return hipGetLastError();
}

hipError_t ctm_svd_left(int count, const cd* const* rho, int n, int k, cd* const* Z, cd* const* ws, hipStream_t st) {
  if (count < 1 || count > CTM_SVD_BATCH || n < 1 || n > CTM_SVD_NMAX || k < 1 || k > n) return hipErrorInvalidValue;
  SvdBatch bt{};
  for (int b = 0; b < count; ++b) {
    bt.rho[b] = rho[b];
    bt.Z[b] = Z[b];
    bt.W[b] = ws[b];
  }
  if (n <= CTM_SVD_REG_NMAX) return launch_svd_reg<1, 2, 2, 1024>(bt, count, n, k, st);
  const int nblk = (n + SVD_MB - 1) / SVD_MB, nb = nblk + (nblk & 1);
  const bool in_lds = n <= SVD_LDS_NMAX;
  const size_t lds = in_lds ? (size_t)2 * SVD_MB * n * sizeof(cd) : 0;
  static bool attr[SVD_ATTR_DEVICES] = {};
  const hipError_t ea = set_lds_attr((const void*)k_ctm_svd_round<true>,
                                     (int)(2 * SVD_MB * SVD_LDS_NMAX * sizeof(cd)), attr);
  if (ea != hipSuccess) return ea;
  hipLaunchKernelGGL(k_ctm_svd_lq, dim3(count), dim3(1024), 0, st, bt, n);
  hipError_t e = hipGetLastError();
  // the first SVD_SWEEPS_FIRST sweeps, then two at a time until a sweep of
  // every matrix made no rotation (the rotation counts read back after each
  // batch: the stream waits there); a sweep after a sweep without rotation
  // returns at once on the device
  int sweep = 0;
  while (e == hipSuccess && sweep < SVD_SWEEPS_MULTI) {
    const int upto = sweep == 0 ? SVD_SWEEPS_FIRST : (sweep + 2 < SVD_SWEEPS_MULTI ? sweep + 2 : SVD_SWEEPS_MULTI);
    for (; sweep < upto && e == hipSuccess; ++sweep)
      for (int r = 0; r < nb - 1 && e == hipSuccess; ++r) {
        if (in_lds)
          hipLaunchKernelGGL(k_ctm_svd_round<true>, dim3(nb / 2, count), dim3(64 * SVD_MB), lds, st, bt, n, nb,
                             sweep, r);
        else
          hipLaunchKernelGGL(k_ctm_svd_round<false>, dim3(nb / 2, count), dim3(64 * SVD_MB), 0, st, bt, n, nb,
                             sweep, r);
        e = hipGetLastError();
      }
    if (e != hipSuccess || sweep >= SVD_SWEEPS_MULTI) break;
    bool done = true;
    for (int b = 0; b < count && e == hipSuccess; ++b) {
      int last = 0;
      const int* rot = (const int*)(ws[b] + (long long)n * n);  // the layout of svd_mem_ws
      e = hipMemcpyAsync(&last, rot + sweep - 1, sizeof(int), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      done = done && last == 0;
    }
    if (done) break;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ctm_svd_final, dim3(count), dim3(256), 0, st, bt, n, k);
  return hipGetLastError();
}

__global__ void k_ctm_ratio(const cd* num, const cd* den, cd* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cd a = num[i], b = den[i];
  const double q = b.x * b.x + b.y * b.y;
  out[i] = cd{(a.x * b.x + a.y * b.y) / q, (a.y * b.x - a.x * b.y) / q};
}

hipError_t ctm_ratio(const cd* num, const cd* den, cd* out, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctm_ratio, dim3((n + 63) / 64), dim3(64), 0, st, num, den, out, n);
  return hipGetLastError();
}

__global__ void k_ctm_sum_ratio(const cd* term, const cd* den, cd* out, int nb, int nt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  cd a{0.0, 0.0};
  for (int t = 0; t < nt; ++t) a += term[b * nt + t];
  const cd d = den[b];
  const double q = d.x * d.x + d.y * d.y;
  out[b] = cd{(a.x * d.x + a.y * d.y) / q, (a.y * d.x - a.x * d.y) / q};
}

hipError_t ctm_sum_ratio(const cd* term, const cd* den, cd* out, int nb, int nt, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctm_sum_ratio, dim3(1), dim3(64), 0, st, term, den, out, nb, nt);
  return hipGetLastError();
}

}  // namespace ntu
