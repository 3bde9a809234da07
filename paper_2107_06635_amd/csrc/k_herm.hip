// Metric repair: the exact metric is Hermitian and non-negative (abstract;
// Sec. II).  Hermitise in place and, on request, clip negative eigenvalues.
#include "kernels.h"
#include "linalg.h"

namespace ntu {

constexpr int HERM_THREADS = 256;
constexpr int HERM_SPLIT = 16;  // workgroups per item
constexpr int CLIP_THREADS = 1024;

// (g + g^H) / 2 in place.  Workgroup (item, b) of HERM_SPLIT takes the b-th
// range of the pairs (i, j), j <= i, so each pair is written by one thread;
// it leaves its partial ||g - g^H||_F^2, ||g||_F^2 and count of non-finite
// input entries in part[item][b] (k_herm_stats adds them up).
template <class T>
__global__ void __launch_bounds__(HERM_THREADS) k_hermitise(int n, T* g, double* part) {
  __shared__ double red[64];
  const int it = blockIdx.x, b = blockIdx.y, nb = gridDim.y;
  T* G = g + (size_t)it * n * n;
  double skew = 0, nrm = 0, bad = 0;
  const long long npair = (long long)n * (n + 1) / 2;
  const long long e0 = npair * b / nb, e1 = npair * (b + 1) / nb;
  for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    // packed lower triangle, row-wise: e -> (i, j), j <= i
    int i = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while ((long long)(i + 1) * (i + 2) / 2 <= e) ++i;
    while ((long long)i * (i + 1) / 2 > e) --i;
    int j = (int)(e - (long long)i * (i + 1) / 2);
    T a = G[(size_t)i * n + j], b = G[(size_t)j * n + i];
    if (!finitev(a)) bad += 1;
    if (i != j && !finitev(b)) bad += 1;
    if (i == j) {
      nrm += abs2(a);
      skew += 4.0 * imv(a) * imv(a);
      G[(size_t)i * n + i] = realv<T>(rev(a));
    } else {
      nrm += abs2(a) + abs2(b);
      T dlt = a - conjv(b);
      skew += 2.0 * abs2(dlt);
      T h = 0.5 * (a + conjv(b));
      G[(size_t)i * n + j] = h;
      G[(size_t)j * n + i] = conjv(h);
    }
  }
  skew = block_sum(skew, red);
  nrm = block_sum(nrm, red);
  bad = block_sum(bad, red);
  if (part && threadIdx.x == 0) {
    double* pp = part + ((size_t)it * nb + b) * 3;
    pp[0] = skew; pp[1] = nrm; pp[2] = bad;
  }
}

// Stats of the Hermitisation from the partial sums: one thread per item.
__global__ void k_herm_stats(int batch, int nb, const double* __restrict__ part, double* stats, int sstride) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= batch) return;
  double skew = 0, nrm = 0, bad = 0;
  for (int b = 0; b < nb; ++b) {
    const double* pp = part + ((size_t)it * nb + b) * 3;
    skew += pp[0]; nrm += pp[1]; bad += pp[2];
  }
  double* s = stats + (size_t)it * sstride;
  s[0] = nrm > 0 ? sqrt(skew) / sqrt(nrm) : 0.0;
  s[1] = sqrt(nrm);
  s[2] = NAN; s[3] = NAN; s[4] = 0.0; s[5] = 0.0;
  s[6] = bad; s[7] = 0.0;
}

// Eigenvalue clip of the Hermitian g.  Rows that are exactly zero are left
// out; if the rest admits a Cholesky factorisation it is positive definite
// and nothing changes; otherwise g <- V max(Lambda, 0) V^H on that block.
// With shift_rel > 0 the tests are first made on g - shift_rel ||g||_F I
// (Gershgorin: lowest disc edge > shift_rel * highest); success there also
// certifies g for the bond fit (cert[it] = 1, else 0; cert may be NULL).
template <class T>
__global__ void __launch_bounds__(CLIP_THREADS) k_clip(int n, T* g, double* stats, int sstride, T* ws,
                                                       double shift_rel, double* cert) {
  __shared__ double red[1024];  // >= blockDim.x (Gershgorin partial sums)
  __shared__ int idx[1024];
  __shared__ int m_sh, cnt;
  __shared__ double pc[512], ps[512];
  __shared__ T pe[512];
  __shared__ int pq[512];
  const int it = blockIdx.x, tid = threadIdx.x;
  T* G = g + (size_t)it * n * n;
  T* A = ws + (size_t)it * 2 * n * n;
  T* V = A + (size_t)n * n;
  // nonzero rows
  for (int i = tid; i < n; i += blockDim.x) {
    bool nz = false;
    for (int j = 0; j < n && !nz; ++j) {
      T v = G[(size_t)i * n + j];
      nz = (rev(v) != 0.0) || (imv(v) != 0.0);
    }
    idx[i] = nz ? 1 : 0;
  }
  __syncthreads();
  if (tid == 0) {
    int m = 0;
    for (int i = 0; i < n; ++i)
      if (idx[i]) idx[m++] = i;
    m_sh = m;
  }
  __syncthreads();
  const int m = m_sh;
  // positive definite (the clip is the identity) if the Gershgorin discs of
  // the full matrix stay right of zero (tested first: it reads g once and
  // needs no copy), or else if a Cholesky factor exists
  if (m == n && gershgorin_certify<T>(G, n, shift_rel, red)) {
    if (cert && tid == 0) cert[it] = 1.0;
    return;
  }
  if (cert && tid == 0) cert[it] = 0.0;
  double fro = 0;
  for (long long e = tid; e < (long long)m * m; e += blockDim.x) {
    int i = (int)(e / m), j = (int)(e % m);
    T v = G[(size_t)idx[i] * n + idx[j]];
    A[e] = v;
    fro += abs2(v);
  }
  fro = sqrt(block_sum(fro, red));
  __syncthreads();
  if (shift_rel > 0.0 && m == n) {
    const double sh = shift_rel * fro;
    for (int i = tid; i < m; i += blockDim.x) A[(size_t)i * m + i] = A[(size_t)i * m + i] - realv<T>(sh);
    __syncthreads();
    if (block_cholesky<T>(A, m, m, red)) {
      if (cert && tid == 0) cert[it] = 1.0;
      return;
    }
    for (long long e = tid; e < (long long)m * m; e += blockDim.x) {
      int i = (int)(e / m), j = (int)(e % m);
      A[e] = G[(size_t)idx[i] * n + idx[j]];
    }
    __syncthreads();
  }
  bool ok = m == 0 || block_cholesky<T>(A, m, m, red);
  if (ok) return;
  for (long long e = tid; e < (long long)m * m; e += blockDim.x) {
    int i = (int)(e / m), j = (int)(e % m);
    A[e] = G[(size_t)idx[i] * n + idx[j]];
  }
  __syncthreads();
  // load batches that keep 1024 threads within 128 VGPRs (no spills)
  const int sweeps = block_jacobi_eigh<T, is_cplx<T>::value ? 3 : 8>(A, m, m, V, m, pc, ps, pe, pq, &cnt, fro);
  // eigenvalues on the diagonal of A
  double lmin = INFINITY, lmax = -INFINITY, neg = 0, tot = 0;
  for (int i = tid; i < m; i += blockDim.x) {
    double l = rev(A[(size_t)i * m + i]);
    lmin = fmin(lmin, l); lmax = fmax(lmax, l);
    if (l < 0) neg -= l;
    tot += fabs(l);
  }
  lmin = -block_max(-lmin, red);
  lmax = block_max(lmax, red);
  neg = block_sum(neg, red);
  tot = block_sum(tot, red);
  // reassemble on the block: G[idx_i, idx_j] = sum_k V[i][k] max(l_k, 0) conj(V[j][k])
  for (long long e = tid; e < (long long)m * m; e += blockDim.x) {
    int i = (int)(e / m), j = (int)(e % m);
    T acc = zerov<T>();
    for (int k = 0; k < m; ++k) {
      double l = rev(A[(size_t)k * m + k]);
      if (l > 0) acc += mulc(V[(size_t)i * m + k], V[(size_t)j * m + k]) * l;
    }
    G[(size_t)idx[i] * n + idx[j]] = acc;
  }
  if (stats && tid == 0) {
    double* s = stats + (size_t)it * sstride;
    s[2] = lmin; s[3] = lmax; s[4] = tot > 0 ? neg / tot : 0.0; s[5] = 1.0; s[7] = sweeps;
  }
}

size_t fix_workspace_bytes(bool cplx, int batch, int n) {
  // the clip's two n x n matrices per item; the Hermitisation's partial sums
  // (batch x HERM_SPLIT x 3 doubles) use the same space first
  const size_t clip = (size_t)batch * 2 * n * n * (cplx ? 16 : 8);
  const size_t part = (size_t)batch * HERM_SPLIT * 3 * sizeof(double);
  return (clip > part ? clip : part) + 256;
}

hipError_t launch_metric_fix(bool cplx, int batch, int n, void* g, int mode, double* stats, int sstride,
                             void* ws, hipStream_t st, const ProfHook& ph, double shift_rel, double* cert) {
  if (batch <= 0) return hipSuccess;
  if (n > 1024) return hipErrorInvalidValue;
  // partial sums at the start of the workspace (read by k_herm_stats before
  // the clip reuses it; same stream)
  double* part = stats ? (double*)ws : nullptr;
  ph(PK_HERM, 0);
  const dim3 hg(batch, HERM_SPLIT);
  if (cplx) hipLaunchKernelGGL(k_hermitise<cd>, hg, dim3(HERM_THREADS), 0, st, n, (cd*)g, part);
  else hipLaunchKernelGGL(k_hermitise<double>, hg, dim3(HERM_THREADS), 0, st, n, (double*)g, part);
  if (stats) hipLaunchKernelGGL(k_herm_stats, dim3((batch + 63) / 64), dim3(64), 0, st, batch, HERM_SPLIT, part, stats, sstride);
  ph(PK_HERM, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || mode == 0) return e;
  ph(PK_CLIP, 0);
  if (cplx)
    hipLaunchKernelGGL(k_clip<cd>, dim3(batch), dim3(CLIP_THREADS), 0, st, n, (cd*)g, stats, sstride, (cd*)ws,
                       shift_rel, cert);
  else
    hipLaunchKernelGGL(k_clip<double>, dim3(batch), dim3(CLIP_THREADS), 0, st, n, (double*)g, stats, sstride,
                       (double*)ws, shift_rel, cert);
  ph(PK_CLIP, 1);
  return hipGetLastError();
}

}  // namespace ntu
