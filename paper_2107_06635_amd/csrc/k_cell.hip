// Gather of the clusters of a group of independent bond updates of a larger
// unit cell into role-major batches, and scatter of the updated X and Y back
// into the cell.  Plain copies (HBM bound), one thread per element.
#include "cell.h"
#include "common.h"

namespace ntu {

template <class T>
__global__ void __launch_bounds__(256) k_cell_gather(const T* __restrict__ cell, T* __restrict__ work, int p, int D,
                                                     CellGroup g) {
  const long long nsite = (long long)p * D * D * D * D;
  const long long total = 8ll * g.n * nsite;
  for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < total;
       o += (long long)gridDim.x * blockDim.x) {
    const long long e = o % nsite, rk = o / nsite;
    const int k = (int)(rk % g.n), r = (int)(rk / g.n);
    long long src = e;
    if (g.vert[k]) {
      // turned clockwise: new (t, l, b, r) = old (l, b, r, t), i.e.
      // out[s][i][j][l][m] = in[s][m][i][j][l]
      long long q = e;
      const int m = (int)(q % D); q /= D;
      const int l = (int)(q % D); q /= D;
      const int j = (int)(q % D); q /= D;
      const int i = (int)(q % D); q /= D;
      const long long s = q;
      src = (((s * D + m) * D + i) * D + j) * D + l;
    }
    work[o] = cell[(long long)g.site[k][r] * nsite + src];
  }
}

template <class T>
__global__ void __launch_bounds__(256) k_cell_scatter(T* __restrict__ cell, const T* __restrict__ work, int p, int D,
                                                      CellGroup g) {
  const long long nsite = (long long)p * D * D * D * D;
  const long long total = 2ll * g.n * nsite;
  for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < total;
       o += (long long)gridDim.x * blockDim.x) {
    const long long e = o % nsite, rk = o / nsite;
    const int k = (int)(rk % g.n), r = (int)(rk / g.n);
    long long dst = e;
    if (g.vert[k]) {
      // turned back (counter-clockwise): work (s, a, b, c, d) is cell
      // (s, d, a, b, c), the inverse of the gather's turn
      long long q = e;
      const int d = (int)(q % D); q /= D;
      const int c = (int)(q % D); q /= D;
      const int b = (int)(q % D); q /= D;
      const int a = (int)(q % D); q /= D;
      const long long s = q;
      dst = (((s * D + d) * D + a) * D + b) * D + c;
    }
    cell[(long long)g.site[k][r] * nsite + dst] = work[o];
  }
}

static int cell_grid(long long n) {
  const long long b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

hipError_t launch_cell_gather(bool cplx, const void* cell, void* work, int p, int D, const CellGroup& g,
                              hipStream_t st) {
  if (g.n < 1 || g.n > CELL_GROUP_MAX) return hipErrorInvalidValue;
  const long long n = 8ll * g.n * p * D * D * D * D;
  if (cplx)
    hipLaunchKernelGGL(k_cell_gather<cd>, dim3(cell_grid(n)), dim3(256), 0, st, (const cd*)cell, (cd*)work, p, D, g);
  else
    hipLaunchKernelGGL(k_cell_gather<double>, dim3(cell_grid(n)), dim3(256), 0, st, (const double*)cell,
                       (double*)work, p, D, g);
  return hipGetLastError();
}

hipError_t launch_cell_scatter(bool cplx, void* cell, const void* work, int p, int D, const CellGroup& g,
                               hipStream_t st) {
  if (g.n < 1 || g.n > CELL_GROUP_MAX) return hipErrorInvalidValue;
  const long long n = 2ll * g.n * p * D * D * D * D;
  if (cplx)
    hipLaunchKernelGGL(k_cell_scatter<cd>, dim3(cell_grid(n)), dim3(256), 0, st, (cd*)cell, (const cd*)work, p, D,
                       g);
  else
    hipLaunchKernelGGL(k_cell_scatter<double>, dim3(cell_grid(n)), dim3(256), 0, st, (double*)cell,
                       (const double*)work, p, D, g);
  return hipGetLastError();
}

}  // namespace ntu
