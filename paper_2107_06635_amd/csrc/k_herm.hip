// Metric repair: the exact metric is Hermitian and non-negative (abstract;
// Sec. II).  Hermitise in place and, on request, clip negative eigenvalues.
#include <utility>
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
                                                       double shift_rel, double* cert, int* need) {
  __shared__ double red[1024];  // >= blockDim.x (Gershgorin partial sums)
  __shared__ int idx[1024];
  __shared__ int m_sh, cnt;
  __shared__ double pc[512], ps[512];
  __shared__ T pe[512];
  __shared__ int pq[512];
  const int it = blockIdx.x, tid = threadIdx.x;
  if (need && tid == 0) need[it] = 0;
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
  // with need, a matrix that fails the tests goes to the sign iteration; the
  // plain Cholesky is left out after a failed shifted one (a positive
  // definite matrix that only misses the certificate comes back from the
  // iteration equal to g up to rounding)
  const bool ok = m == 0 || ((!need || shift_rel <= 0.0 || m < n) && block_cholesky<T>(A, m, m, red));
  if (ok) return;
  if (need) {
    if (tid == 0) need[it] = 1;
    return;
  }
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

// ---------------------------------------------------------------------------
// Clip by the matrix sign function (real g, n >= NS_MIN_N).  With S = sign(g)
// (eigenvalues +-1 on the eigenvectors of g), max(Lambda, 0) on the same
// vectors is (g + g S) / 2.  S comes from a polynomial iteration on X = g /
// ||g||_F (all eigenvalues in [-1, 1]) that only multiplies matrices, on the
// FP64 matrix cores over the whole chip:
//   NS_K1 steps X <- X (a I + b X^2 + c X^4), (a, b, c) = (3.4445, -4.7750,
//   2.0315): an odd quintic that multiplies eigenvalues below 0.1 by about
//   3.44 and maps [0, 1.2024] into [0, 1.2024], every value above 0.3 into
//   [0.68, 1.2024];
//   NS_K2 steps X <- (3 X - X^3) / 2 (Newton-Schulz), which takes [0.68,
//   1.2024] to 1 quadratically (six steps from 0.68 reach 1 - 1e-16) and
//   keeps (0, sqrt 3) inside (0, 1].
// Every eigenvalue of magnitude >= 1e-15 ||g||_F reaches sign +-1 to
// rounding; a smaller one ends with |s| <= 1, so its contribution
// lambda (1 + s) / 2 lies between 0 and lambda: the result is within that
// size of V max(Lambda, 0) V^T (measured 3e-15 relative at n = 400 for a
// spectrum with 300 eigenvalues of +-1e-7).
// ---------------------------------------------------------------------------
constexpr int NS_MIN_N = 128;
constexpr int NS_K1 = 28, NS_K2 = 6;
constexpr double NS_A = 3.4445, NS_B = -4.7750, NS_C = 2.0315;
constexpr int NS_T = 32;  // tile of the products

// C = alpha A B + beta E + gamma I for square row-major n x n matrices of
// the items with need[item] != 0 (item strides sa, sb, se, sc elements; E may
// be NULL; C must not alias A, B or E).  Workgroup: one 32 x 32 tile of one
// item (blockIdx.z), four waves of 16 x 16 on v_mfma_f64_16x16x4 (lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16] of each 16 x 4 x 16 step and
// receives C[l / 16 + 4 v][l % 16]); K in chunks of 32 through shared
// memory, loaded from clamped addresses and masked when stored.
__global__ void __launch_bounds__(256) k_ns_gemm(int n, const double* __restrict__ A, long long sa,
                                                 const double* __restrict__ B, long long sb,
                                                 const double* __restrict__ E, long long se, double* __restrict__ C,
                                                 long long sc, double alpha, double beta, double gamma,
                                                 const int* __restrict__ need) {
  const int it = blockIdx.z;
  if (!need[it]) return;
  __shared__ double As[NS_T][NS_T + 1];  // [row][k]
  __shared__ double Bs[NS_T][NS_T + 1];  // [k][col]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int i0 = blockIdx.y * NS_T, j0 = blockIdx.x * NS_T;
  const int wr = (w >> 1) * 16, wc = (w & 1) * 16;
  const double* Ab = A + it * sa;
  const double* Bb = B + it * sb;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < n; k0 += NS_T) {
    double va[4], vb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u, r = e >> 5, c = e & 31;
      va[u] = Ab[min(i0 + r, n - 1) * n + min(k0 + c, n - 1)];
      vb[u] = Bb[min(k0 + r, n - 1) * n + min(j0 + c, n - 1)];
    }
    __syncthreads();  // the previous chunk's fragments have been read
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u, r = e >> 5, c = e & 31;
      As[r][c] = (i0 + r < n && k0 + c < n) ? va[u] : 0.0;
      Bs[r][c] = (k0 + r < n && j0 + c < n) ? vb[u] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kc = 0; kc < NS_T / 4; ++kc)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[wr + l16][4 * kc + lk], Bs[4 * kc + lk][wc + l16], acc, 0, 0, 0);
  }
  double* Cb = C + it * sc;
  const double* Eb = E ? E + it * se : nullptr;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + wr + lk + 4 * v, j = j0 + wc + l16;
    if (i < n && j < n) {
      double val = alpha * acc[v];
      if (Eb) val += beta * Eb[i * n + j];
      if (i == j) val += gamma;
      Cb[i * n + j] = val;
    }
  }
}

// X = g / ||g||_F for the items that need the iteration; tr[item] = trace(g).
__global__ void __launch_bounds__(1024) k_ns_init(int n, const double* __restrict__ g, double* __restrict__ X,
                                                  long long sx, double* __restrict__ tr, const int* __restrict__ need) {
  __shared__ double red[64];
  const int it = blockIdx.x;
  if (!need[it]) return;
  const double* G = g + (size_t)it * n * n;
  double* Xi = X + it * sx;
  const int nn = n * n;
  double f = 0.0, t = 0.0;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const double v = G[e];
    f += v * v;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) t += G[i * n + i];
  f = block_sum(f, red);
  t = block_sum(t, red);
  const double inv = f > 0.0 ? 1.0 / sqrt(f) : 0.0;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) Xi[e] = G[e] * inv;
  if (threadIdx.x == 0) tr[it] = t;
}

// g = (P + P^T) / 2 from P = (g + g S) / 2, and the stats of the clip:
// trace |g| = trace(g S) = 2 trace P - trace g, clipped mass (sum of -lambda
// over negative lambda) / sum |lambda| = (trace P - trace g) / (2 trace P -
// trace g).  Grid (batch, HERM_SPLIT): rows split over the workgroups.
__global__ void __launch_bounds__(256) k_ns_finish(int n, double* __restrict__ g, const double* __restrict__ P,
                                                   long long sp, const double* __restrict__ tr, double* stats,
                                                   int sstride, const int* __restrict__ need) {
  __shared__ double red[64];
  const int it = blockIdx.x;
  if (!need[it]) return;
  double* G = g + (size_t)it * n * n;
  const double* Pi = P + it * sp;
  const int rows = (n + gridDim.y - 1) / gridDim.y, r0 = blockIdx.y * rows, r1 = min(n, r0 + rows);
  for (int e = threadIdx.x; e < (r1 - r0) * n; e += blockDim.x) {
    const int i = r0 + e / n, j = e % n;
    G[i * n + j] = 0.5 * (Pi[i * n + j] + Pi[j * n + i]);
  }
  if (stats && blockIdx.y == 0) {
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) t += Pi[i * n + i];
    t = block_sum(t, red);
    if (threadIdx.x == 0) {
      double* s = stats + (size_t)it * sstride;
      const double den = 2.0 * t - tr[it];
      s[2] = NAN; s[3] = NAN; s[4] = den > 0.0 ? (t - tr[it]) / den : 0.0; s[5] = 2.0; s[7] = NS_K1 + NS_K2;
    }
  }
}

static bool use_sign_clip(bool cplx, int n) { return !cplx && n >= NS_MIN_N; }

// the sign iteration's three matrices per item, then the flags and traces
static size_t ns_matrix_bytes(int batch, int n) { return (size_t)batch * 3 * n * n * sizeof(double); }

size_t fix_workspace_bytes(bool cplx, int batch, int n) {
  // the clip's two n x n matrices per item (three for the sign iteration,
  // then its per-item flags and traces); the Hermitisation's partial sums
  // (batch x HERM_SPLIT x 3 doubles) use the same space first
  const size_t clip = use_sign_clip(cplx, n) ? ns_matrix_bytes(batch, n) + (size_t)batch * 16 + 256
                                             : (size_t)batch * 2 * n * n * (cplx ? 16 : 8);
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
  if (cplx) {
    hipLaunchKernelGGL(k_clip<cd>, dim3(batch), dim3(CLIP_THREADS), 0, st, n, (cd*)g, stats, sstride, (cd*)ws,
                       shift_rel, cert, (int*)nullptr);
  } else if (!use_sign_clip(cplx, n)) {
    hipLaunchKernelGGL(k_clip<double>, dim3(batch), dim3(CLIP_THREADS), 0, st, n, (double*)g, stats, sstride,
                       (double*)ws, shift_rel, cert, (int*)nullptr);
  } else {
    // certificate tests first (they use the start of the workspace), then the
    // sign iteration for the items they leave; the three matrices of item i
    // at ws + 3 n^2 i, the flags and traces after all of them
    double* base = (double*)ws;
    const long long nn = (long long)n * n, sm = 3 * nn;
    char* tail = (char*)ws + ns_matrix_bytes(batch, n);
    int* need = (int*)tail;
    double* tr = (double*)(tail + (((size_t)batch * sizeof(int) + 15) & ~(size_t)15));
    hipLaunchKernelGGL(k_clip<double>, dim3(batch), dim3(CLIP_THREADS), 0, st, n, (double*)g, stats, sstride,
                       base, shift_rel, cert, need);
    double* M[3] = {base, base + nn, base + 2 * nn};
    hipLaunchKernelGGL(k_ns_init, dim3(batch), dim3(1024), 0, st, n, (const double*)g, M[0], sm, tr, (const int*)need);
    const int tiles = (n + NS_T - 1) / NS_T;
    const dim3 gg(tiles, tiles, batch);
    auto gemm = [&](const double* A, long long sa, const double* B, const double* E, long long se, double* C,
                    double alpha, double beta, double gamma) {
      hipLaunchKernelGGL(k_ns_gemm, gg, dim3(256), 0, st, n, A, sa, B, sm, E, se, C, sm, alpha, beta, gamma,
                         (const int*)need);
    };
    int x = 0, y = 1, w = 2;
    for (int k = 0; k < NS_K1; ++k) {
      gemm(M[x], sm, M[x], nullptr, 0, M[y], 1.0, 0.0, 0.0);        // Y = X^2
      gemm(M[y], sm, M[y], M[y], sm, M[w], NS_C, NS_B, NS_A);       // W = a I + b Y + c Y^2
      gemm(M[x], sm, M[w], nullptr, 0, M[y], 1.0, 0.0, 0.0);        // X <- X W
      std::swap(x, y);
    }
    for (int k = 0; k < NS_K2; ++k) {
      gemm(M[x], sm, M[x], nullptr, 0, M[y], 1.0, 0.0, 0.0);        // Y = X^2
      gemm(M[x], sm, M[y], M[x], sm, M[w], -0.5, 1.5, 0.0);         // X <- 3/2 X - 1/2 X Y
      std::swap(x, w);
    }
    // P = (g + g S) / 2 into a free matrix, then g = (P + P^T) / 2
    gemm((const double*)g, nn, M[x], (const double*)g, nn, M[y], 0.5, 0.5, 0.0);
    hipLaunchKernelGGL(k_ns_finish, dim3(batch, HERM_SPLIT), dim3(256), 0, st, n, (double*)g, (const double*)M[y],
                       sm, (const double*)tr, stats, sstride, (const int*)need);
  }
  ph(PK_CLIP, 1);
  return hipGetLastError();
}

}  // namespace ntu
