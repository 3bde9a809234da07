// Device primitives of the CTMRG expectation values: permutation of tensor
// axes, complex products, normalisation by the largest modulus, and the
// leading eigenvectors of a Hermitian matrix (the isometry of a cut).
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
__global__ void __launch_bounds__(256) k_ctm_gemm(const cd* __restrict__ A, const cd* __restrict__ B,
                                                  cd* __restrict__ C, int M, int N, int K) {
  constexpr int T = 32, KC = 16;
  __shared__ cd As[KC][T + 1];
  __shared__ cd Bs[KC][T + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * T, j0 = blockIdx.x * T;
  cd acc[2][2] = {{cd{0, 0}, cd{0, 0}}, {cd{0, 0}, cd{0, 0}}};
  for (int k0 = 0; k0 < K; k0 += KC) {
    for (int e = tid; e < KC * T; e += 256) {
      const int r = e / KC, kk = e % KC;            // A: row r of the tile, column kk of the chunk
      const int i = i0 + r, k = k0 + kk;
      As[kk][r] = (i < M && k < K) ? A[(long long)i * K + k] : cd{0, 0};
      const int kb = e / T, c = e % T;              // B: row kb of the chunk, column c of the tile
      const int kk2 = k0 + kb, j = j0 + c;
      Bs[kb][c] = (kk2 < K && j < N) ? B[(long long)kk2 * N + j] : cd{0, 0};
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

hipError_t ctm_gemm(const cd* A, const cd* B, cd* C, int M, int N, int K, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 g((N + 31) / 32, (M + 31) / 32);
  hipLaunchKernelGGL(k_ctm_gemm, g, dim3(256), 0, st, A, B, C, M, N, K);
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

// Leading left singular vectors of an n x n matrix rho without squaring its
// singular values: the Hermitian matrix [[0, rho], [rho^H, 0]] (2n x 2n) has
// the eigenvalues +-sigma_i with eigenvectors (u_i, +-v_i) / sqrt(2), so its
// k largest eigenvalues give u_1..u_k, resolved down to rounding relative to
// sigma_1 (the eigenproblem of rho rho^H would lose the singular values
// below sqrt(eps) sigma_1).  Cyclic Jacobi on the 2n matrix (copied into A,
// eigenvectors into V), the upper halves of the k leading eigenvectors times
// sqrt(2) into Z, then Gram-Schmidt twice over Z's columns; a column with
// nothing left after the projections (rho of rank below k) is replaced by
// the first unit vector that leaves something, so Z always has orthonormal
// columns.  One workgroup.
__global__ void __launch_bounds__(1024) k_ctm_svd_left(const cd* __restrict__ rho, int n, int k, cd* __restrict__ Z,
                                                       cd* __restrict__ A, cd* __restrict__ V) {
  constexpr int NM = 2 * CTM_SVD_NMAX;
  __shared__ double pc[NM / 2 + 1], ps[NM / 2 + 1];
  __shared__ cd pe[NM / 2 + 1];
  __shared__ int pq[NM / 2 + 1];
  __shared__ int cnt, pick_sh;
  __shared__ double lam[NM];
  __shared__ double red[64];
  __shared__ int rank_of[NM];
  const int tid = threadIdx.x, m = 2 * n;
  double fro = 0.0;
  for (long long e = tid; e < (long long)m * m; e += blockDim.x) {
    const int i = (int)(e / m), j = (int)(e % m);
    cd v{0.0, 0.0};
    if (i < n && j >= n) v = rho[(long long)i * n + (j - n)];
    else if (i >= n && j < n) v = conjv(rho[(long long)j * n + (i - n)]);
    A[e] = v;
    fro += abs2(v);
  }
  fro = sqrt(block_sum(fro, red));
  __syncthreads();
  block_jacobi_eigh<cd>(A, m, m, V, m, pc, ps, pe, pq, &cnt, fro);
  for (int i = tid; i < m; i += blockDim.x) lam[i] = A[(long long)i * m + i].x;
  __syncthreads();
  for (int i = tid; i < m; i += blockDim.x) {
    int r = 0;
    for (int j = 0; j < m; ++j) r += (lam[j] > lam[i] || (lam[j] == lam[i] && j < i)) ? 1 : 0;
    rank_of[i] = r;
  }
  __syncthreads();
  const double sq2 = sqrt(2.0);
  for (long long e = tid; e < (long long)n * m; e += blockDim.x) {
    const int row = (int)(e / m), col = (int)(e % m);
    const int r = rank_of[col];
    if (r < k) Z[(long long)row * k + r] = V[(long long)row * m + col] * sq2;
  }
  __syncthreads();
  // Gram-Schmidt twice, column by column, with completion
  int next_unit = 0;
  for (int c = 0; c < k; ++c) {
    for (int attempt = 0; attempt <= n; ++attempt) {
      for (int pass = 0; pass < 2; ++pass)
        for (int b = 0; b < c; ++b) {
          cd dot{0.0, 0.0};
          for (int i = tid; i < n; i += blockDim.x) dot += cmul(Z[(long long)i * k + b], Z[(long long)i * k + c]);
          dot.x = block_sum(dot.x, red);
          dot.y = block_sum(dot.y, red);
          for (int i = tid; i < n; i += blockDim.x)
            Z[(long long)i * k + c] = Z[(long long)i * k + c] - dot * Z[(long long)i * k + b];
          __syncthreads();
        }
      double nn = 0.0;
      for (int i = tid; i < n; i += blockDim.x) nn += abs2(Z[(long long)i * k + c]);
      nn = sqrt(block_sum(nn, red));
      if (nn > 0.5) {
        const double inv = 1.0 / nn;
        for (int i = tid; i < n; i += blockDim.x) Z[(long long)i * k + c] = Z[(long long)i * k + c] * inv;
        __syncthreads();
        break;
      }
      // nothing independent left: try the next unit vector
      if (tid == 0) pick_sh = next_unit;
      __syncthreads();
      const int u = pick_sh;
      for (int i = tid; i < n; i += blockDim.x) Z[(long long)i * k + c] = cd{i == u ? 1.0 : 0.0, 0.0};
      ++next_unit;
      __syncthreads();
    }
  }
}

hipError_t ctm_svd_left(const cd* rho, int n, int k, cd* Z, cd* ws, hipStream_t st) {
  if (n < 1 || n > CTM_SVD_NMAX || k < 1 || k > n) return hipErrorInvalidValue;
  const long long m = 2ll * n;
  hipLaunchKernelGGL(k_ctm_svd_left, dim3(1), dim3(1024), 0, st, rho, n, k, Z, ws, ws + m * m);
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
