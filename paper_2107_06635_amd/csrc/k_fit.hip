// Bond fit (Fig. 5, Eqs. (2)-(5)): SVDU guess, alternating least squares with
// tilting and a tolerance-selected pseudo-inverse, final balancing.
// One workgroup per bond; the whole loop runs on the device.
//
// Solve of a half-step.  The pseudo-inverse of Eq. (4) is taken at the
// tolerance (from an ascending ladder, relative to the largest eigenvalue)
// that minimises the directly evaluated error of Eq. (2); near-ties go to the
// larger tolerance.  When a Cholesky factor certifies
//     lambda_min >= 1 / tr(g_s^{-1}) > 10 * tol_max * ||g_s||_F >= 10 * tol_max * lambda_max,
// no ladder value removes an eigenvalue, every candidate is the plain
// inverse, and the largest tolerance wins the tie: the solution is
// L^{-H} L^{-1} J with no eigendecomposition.  Otherwise the Jacobi
// eigendecomposition evaluates the ladder.  Rows of g_s that are exactly
// zero (dependent directions) are removed first in both cases.
#include "kernels.h"
#include "linalg.h"

namespace ntu {

constexpr int FIT_THREADS = 512;
constexpr int FIT_RMAX = 20;


// per-item global workspace (elements of T)
NTU_HD long long fit_ws_elems(int D, int R) {
  long long n = (long long)R * R, nx = (long long)R * D;
  return n * nx      // G1
         + 3 * nx * nx  // g_s, A (Cholesky / eigen), X (inverse / eigenvectors)
         + 3 * n;       // g y, d, g d
}

size_t fit_workspace_bytes(bool cplx, int batch, int D, int R) {
  return (size_t)batch * fit_ws_elems(D, R) * (cplx ? 16 : 8) + 256;
}

template <class T> struct FitShared {
  T* y;    // R^2          vec(P)
  T* MX;   // R x D        row-major
  T* MY;   // R x D
  T* Qf;   // R x D        isometric factor of the current half-step
  T* J;    // R D
  T* m;    // R D
  T* sa;   // R x R        column-major SVD work
  T* sv;   // R x R
  double* s;    // R
  int* idx;     // R D
  double* red;  // 16 * 64
  double* vec;  // 64
};

// out[r] = sum_c g[r][c] v[c] for r < n: one wave per row, lanes over columns.
template <class T>
NTU_DEV void fit_matvec(const T* __restrict__ g, int n, const T* v, T* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int r = w; r < n; r += nw) {
    const T* gr = g + (size_t)r * n;
    T acc = zerov<T>();
    for (int c = lane; c < n; c += 64) acc += gr[c] * v[c];
    acc = wave_sum(acc);
    if (lane == 0) out[r] = acc;
  }
}

// d = vec(MX MY^T) - y ; eps = Re(d^H g d).  Whole block.
template <class T>
NTU_DEV double fit_error(const T* __restrict__ g, int R, int Dn, const FitShared<T>& S, T* d, T* gd) {
  const int n = R * R;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    int a = e / R, b = e % R;
    T v = zerov<T>();
    for (int j = 0; j < Dn; ++j) v += S.MX[a * FIT_RMAX + j] * S.MY[b * FIT_RMAX + j];
    d[e] = v - S.y[e];
  }
  __syncthreads();
  fit_matvec<T>(g, n, d, gd);
  __syncthreads();
  double acc = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x) acc += rev(cmul(d[r], gd[r]));
  return block_sum(acc, S.red);
}

// Gram-Schmidt (projection twice) of the columns of M (R x Dn, row-major with
// stride FIT_RMAX) into Q; dependent columns become exactly zero.  Wave 0.
template <class T>
NTU_DEV void fit_orthonormalise(const T* M, T* Q, int R, int Dn, double kappa) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  double scale = 0;
  for (int j = 0; j < Dn; ++j) {
    double v = lane < R ? abs2(M[lane * FIT_RMAX + j]) : 0.0;
    scale = fmax(scale, sqrt(wave_sum(v)));
  }
  for (int j = 0; j < Dn; ++j) {
    T v = lane < R ? M[lane * FIT_RMAX + j] : zerov<T>();
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        T qi = lane < R ? Q[lane * FIT_RMAX + i] : zerov<T>();
        T h = wave_sum(cmul(qi, v));
        v -= qi * h;
      }
    double nn = sqrt(wave_sum(abs2(v)));
    double inv = (scale > 0 && nn > kappa * scale) ? 1.0 / nn : 0.0;
    if (lane < R) Q[lane * FIT_RMAX + j] = v * inv;
  }
}

// Solve the half-step system gs m = J (see the file comment).  gs: nx x nx in
// global memory.  Returns the chosen tolerance; *used_eig = 1 if the ladder
// was evaluated through the eigendecomposition.  `eval(m)` must return the
// error of candidate m (whole-block call).
template <class T, class Eval>
NTU_DEV double fit_solve(const T* gs, int nx, const FitParams& fp, const FitShared<T>& S, T* A, T* X,
                         double N, int* used_eig, Eval eval) {
  __shared__ int m_sh, cnt;
  __shared__ double pc[256], ps[256];
  __shared__ T pe[256];
  const int tid = threadIdx.x;
  // exactly-zero rows
  for (int i = tid; i < nx; i += blockDim.x) {
    bool nz = false;
    for (int j = 0; j < nx && !nz; ++j) {
      T v = gs[(size_t)i * nx + j];
      nz = (rev(v) != 0.0) || (imv(v) != 0.0);
    }
    S.idx[i] = nz ? 1 : 0;
  }
  __syncthreads();
  if (tid == 0) {
    int m = 0;
    for (int i = 0; i < nx; ++i)
      if (S.idx[i]) S.idx[m++] = i;
    m_sh = m;
  }
  __syncthreads();
  const int m = m_sh;
  const double tol_max = fp.tol[fp.n_tol - 1];
  for (int i = tid; i < nx; i += blockDim.x) S.m[i] = zerov<T>();
  double fro = 0;
  for (long long e = tid; e < (long long)m * m; e += blockDim.x) {
    T v = gs[(size_t)S.idx[e / m] * nx + S.idx[e % m]];
    A[e] = v;
    fro += abs2(v);
  }
  fro = sqrt(block_sum(fro, S.red));
  __syncthreads();
  *used_eig = 0;
  if (m == 0) return tol_max;
  bool chol = block_cholesky<T>(A, m, m, S.red);
  if (chol) {
    // X = L^{-1} (lower triangular), row by row
    for (int i = 0; i < m; ++i) {
      for (int j = tid; j <= i; j += blockDim.x) {
        T v;
        if (j == i) v = realv<T>(1.0 / rev(A[(size_t)i * m + i]));
        else {
          T acc = zerov<T>();
          for (int k = j; k < i; ++k) acc += A[(size_t)i * m + k] * X[(size_t)k * m + j];
          v = -acc * (1.0 / rev(A[(size_t)i * m + i]));
        }
        X[(size_t)i * m + j] = v;
      }
      __syncthreads();
    }
    double tr = 0;
    for (long long e = tid; e < (long long)m * m; e += blockDim.x)
      if (e % m <= e / m) tr += abs2(X[e]);
    tr = block_sum(tr, S.red);
    if (tr > 0 && 1.0 / tr > 10.0 * tol_max * fro) {
      // m = X^H (X J)
      T* z = A;  // the factor is no longer needed; reuse its first row
      for (int i = tid; i < m; i += blockDim.x) {
        T acc = zerov<T>();
        for (int j = 0; j <= i; ++j) acc += X[(size_t)i * m + j] * S.J[S.idx[j]];
        z[i] = acc;
      }
      __syncthreads();
      for (int j = tid; j < m; j += blockDim.x) {
        T acc = zerov<T>();
        for (int i = j; i < m; ++i) acc += cmul(X[(size_t)i * m + j], z[i]);
        S.m[S.idx[j]] = acc;
      }
      __syncthreads();
      return tol_max;
    }
  }
  // eigendecomposition ladder
  *used_eig = 1;
  for (long long e = tid; e < (long long)m * m; e += blockDim.x)
    A[e] = gs[(size_t)S.idx[e / m] * nx + S.idx[e % m]];
  __syncthreads();
  block_jacobi_eigh<T>(A, m, m, X, m, pc, ps, pe, &cnt, fro);
  double lmax = -INFINITY;
  for (int i = tid; i < m; i += blockDim.x) lmax = fmax(lmax, rev(A[(size_t)i * m + i]));
  lmax = block_max(lmax, S.red);
  if (!(lmax > 0.0)) return tol_max;  // nothing positive to invert: m = 0
  __shared__ T proj[256];
  for (int i = tid; i < m; i += blockDim.x) {
    T acc = zerov<T>();
    for (int r = 0; r < m; ++r) acc += cmul(X[(size_t)r * m + i], S.J[S.idx[r]]);
    proj[i] = acc;
  }
  __syncthreads();
  // candidate errors for each ladder tolerance (identical kept sets share one evaluation)
  double errs[16];
  int prev_keep = -1;
  double prev_err = 0;
  for (int t = 0; t < fp.n_tol; ++t) {
    double thr = fp.tol[t] * lmax;
    int keep = 0;
    for (int i = 0; i < m; ++i) keep += rev(A[(size_t)i * m + i]) > thr ? 1 : 0;
    if (keep == prev_keep) { errs[t] = prev_err; continue; }
    for (int r = tid; r < m; r += blockDim.x) {
      T acc = zerov<T>();
      for (int i = 0; i < m; ++i) {
        double l = rev(A[(size_t)i * m + i]);
        if (l > thr) acc += X[(size_t)r * m + i] * proj[i] * (1.0 / l);
      }
      S.m[S.idx[r]] = acc;
    }
    __syncthreads();
    prev_err = eval(S.m);
    prev_keep = keep;
    errs[t] = prev_err;
  }
  double emin = INFINITY;
  for (int t = 0; t < fp.n_tol; ++t) emin = fmin(emin, errs[t]);
  int best = 0;
  for (int t = 0; t < fp.n_tol; ++t)
    if (errs[t] <= emin + fp.tie * N) best = t;
  // rebuild the chosen candidate
  double thr = fp.tol[best] * lmax;
  for (int r = tid; r < m; r += blockDim.x) {
    T acc = zerov<T>();
    for (int i = 0; i < m; ++i) {
      double l = rev(A[(size_t)i * m + i]);
      if (l > thr) acc += X[(size_t)r * m + i] * proj[i] * (1.0 / l);
    }
    S.m[S.idx[r]] = acc;
  }
  __syncthreads();
  return fp.tol[best];
}

template <class T>
__global__ void __launch_bounds__(FIT_THREADS) k_bond_fit(int D, int R, const T* __restrict__ g,
                                                          const T* __restrict__ RX, const T* __restrict__ RY,
                                                          FitParams fp, T* MXo, T* MYo, double* stats,
                                                          int stats_stride, T* ws) {
  extern __shared__ double shmem[];
  __shared__ int flag;
  const int it = blockIdx.x, tid = threadIdx.x;
  const int n = R * R;
  const T* G = g + (size_t)it * n * n;
  T* W = ws + (size_t)it * fit_ws_elems(D, R);
  T* G1 = W;
  T* gs = G1 + (size_t)n * R * D;
  T* A = gs + (size_t)R * D * R * D;
  T* X = A + (size_t)R * D * R * D;
  T* gy = X + (size_t)R * D * R * D;
  T* dv = gy + n;
  T* gd = dv + n;
  // shared carve-up
  FitShared<T> S;
  {
    T* p = (T*)shmem;
    S.y = p; p += n;
    S.MX = p; p += FIT_RMAX * FIT_RMAX;
    S.MY = p; p += FIT_RMAX * FIT_RMAX;
    S.Qf = p; p += FIT_RMAX * FIT_RMAX;
    S.J = p; p += FIT_RMAX * FIT_RMAX;
    S.m = p; p += FIT_RMAX * FIT_RMAX;
    S.sa = p; p += FIT_RMAX * FIT_RMAX;
    S.sv = p; p += FIT_RMAX * FIT_RMAX;
    double* q = (double*)p;
    S.s = q; q += FIT_RMAX;
    S.red = q; q += 16 * 64;
    S.vec = q; q += 64;
    S.idx = (int*)q;
  }
  double* st = stats ? stats + (size_t)it * stats_stride : nullptr;
  const double kappa = fp.kappa;

  // P = RX RY^T  (column-major copy in sa for the SVD, row-major y = vec(P))
  for (int e = tid; e < n; e += blockDim.x) {
    int a = e / R, b = e % R;
    T v = zerov<T>();
    for (int k = 0; k < R; ++k) v += RX[(size_t)it * n + a * R + k] * RY[(size_t)it * n + b * R + k];
    S.y[e] = v;
    S.sa[a + b * FIT_RMAX] = v;
  }
  __syncthreads();
  svd_block_small<T>(S.sa, R, R, FIT_RMAX, S.sv, FIT_RMAX, S.s, &flag);
  const double s0 = S.s[0];
  int Dn = 0;
  if (s0 > 0)
    for (int j = 0; j < R && Dn < D; ++j)
      if (S.s[j] > kappa * s0) ++Dn;
  // SVDU: MX = U S^1/2 (columns of sa are U s), MY = conj(V) S^1/2
  for (int e = tid; e < R * FIT_RMAX; e += blockDim.x) {
    int a = e / FIT_RMAX, j = e % FIT_RMAX;
    T mx = zerov<T>(), my = zerov<T>();
    if (j < Dn) {
      double sq = sqrt(S.s[j]);
      mx = S.sa[a + j * FIT_RMAX] * (1.0 / sq);
      my = conjv(S.sv[a + j * FIT_RMAX]) * sq;
    }
    S.MX[e] = mx;
    S.MY[e] = my;
  }
  // g y and N
  __syncthreads();
  fit_matvec<T>(G, n, S.y, gy);
  __syncthreads();
  double N = 0;
  for (int r = tid; r < n; r += blockDim.x) N += rev(cmul(S.y[r], gy[r]));
  N = block_sum(N, S.red);
  double eps = Dn > 0 ? fit_error<T>(G, R, Dn, S, dv, gd) : 0.0;
  if (st && tid == 0) {
    const int len = fit_stats_len(fp.n_iter, D);
    for (int i = 0; i < len; ++i) st[i] = 0.0;
    st[0] = N; st[1] = eps; st[4] = Dn;
  }
  __syncthreads();
  int iters = 0, n_eig = 0;
  double prev = eps;
  for (int iter = 0; iter < fp.n_iter && Dn > 0; ++iter) {
    for (int half = 0; half < 2; ++half) {
      // fixed factor F (MY for the X half-step, MX for the Y half-step), made isometric
      const T* F = half == 0 ? S.MY : S.MX;
      fit_orthonormalise<T>(F, S.Qf, R, Dn, kappa);
      __syncthreads();
      const int nx = R * Dn;
      // G1[(a' b'), c] :  X half: c = (a, j): sum_b g[(a' b'), (a b)] Q[b, j]
      //                   Y half: c = (j, b): sum_a g[(a' b'), (a b)] Q[a, j]
      for (long long e = tid; e < (long long)n * nx; e += blockDim.x) {
        int row = (int)(e / nx), c = (int)(e % nx);
        const T* gr = G + (size_t)row * n;
        T v = zerov<T>();
        if (half == 0) {
          int a = c / Dn, j = c % Dn;
          for (int b = 0; b < R; ++b) v += gr[a * R + b] * S.Qf[b * FIT_RMAX + j];
        } else {
          int j = c / R, b = c % R;
          for (int a = 0; a < R; ++a) v += gr[a * R + b] * S.Qf[a * FIT_RMAX + j];
        }
        G1[e] = v;
      }
      __syncthreads();
      // g_s[r, c] = sum conj(Q) G1 ;  J[r] = sum conj(Q) g y
      for (long long e = tid; e < (long long)nx * nx; e += blockDim.x) {
        int r = (int)(e / nx), c = (int)(e % nx);
        T v = zerov<T>();
        if (half == 0) {
          int ap = r / Dn, jp = r % Dn;
          for (int bp = 0; bp < R; ++bp) v += cmul(S.Qf[bp * FIT_RMAX + jp], G1[(size_t)(ap * R + bp) * nx + c]);
        } else {
          int jp = r / R, bp = r % R;
          for (int ap = 0; ap < R; ++ap) v += cmul(S.Qf[ap * FIT_RMAX + jp], G1[(size_t)(ap * R + bp) * nx + c]);
        }
        gs[e] = v;
      }
      for (int r = tid; r < nx; r += blockDim.x) {
        T v = zerov<T>();
        if (half == 0) {
          int ap = r / Dn, jp = r % Dn;
          for (int bp = 0; bp < R; ++bp) v += cmul(S.Qf[bp * FIT_RMAX + jp], gy[ap * R + bp]);
        } else {
          int jp = r / R, bp = r % R;
          for (int ap = 0; ap < R; ++ap) v += cmul(S.Qf[ap * FIT_RMAX + jp], gy[ap * R + bp]);
        }
        S.J[r] = v;
      }
      __syncthreads();
      // candidate -> free factor, then error
      auto set_free = [&](const T* mv) {
        for (int e = tid; e < R * Dn; e += blockDim.x) {
          if (half == 0) {
            int a = e / Dn, j = e % Dn;
            S.MX[a * FIT_RMAX + j] = mv[a * Dn + j];
            S.MY[a * FIT_RMAX + j] = S.Qf[a * FIT_RMAX + j];
          } else {
            int j = e / R, b = e % R;
            S.MY[b * FIT_RMAX + j] = mv[j * R + b];
            S.MX[b * FIT_RMAX + j] = S.Qf[b * FIT_RMAX + j];
          }
        }
        __syncthreads();
      };
      auto eval = [&](const T* mv) -> double {
        set_free(mv);
        return fit_error<T>(G, R, Dn, S, dv, gd);
      };
      int used_eig = 0;
      double tau = fit_solve<T>(gs, nx, fp, S, A, X, N, &used_eig, eval);
      set_free(S.m);
      eps = fit_error<T>(G, R, Dn, S, dv, gd);
      n_eig += used_eig;
      if (st && tid == 0) {
        st[16 + 2 * iter + half] = eps;
        st[16 + 2 * fp.n_iter + 2 * iter + half] = tau;
      }
    }
    iters = iter + 1;
    bool stop = fp.early_stop && (prev - eps <= fp.conv_tol * N);
    prev = eps;
    if (stop) break;
  }
  __syncthreads();
  // balance: SVD of MX MY^T, normalise by the largest singular value
  for (int e = tid; e < R * R; e += blockDim.x) {
    int a = e % R, b = e / R;
    T v = zerov<T>();
    for (int j = 0; j < Dn; ++j) v += S.MX[a * FIT_RMAX + j] * S.MY[b * FIT_RMAX + j];
    S.sa[a + b * FIT_RMAX] = v;
  }
  __syncthreads();
  svd_block_small<T>(S.sa, R, R, FIT_RMAX, S.sv, FIT_RMAX, S.s, &flag);
  const double c0 = S.s[0];
  int Dk = 0;
  if (c0 > 0)
    for (int j = 0; j < R && Dk < D; ++j)
      if (S.s[j] > kappa * c0) ++Dk;
  if (Dk > Dn) Dk = Dn;
  for (int e = tid; e < R * D; e += blockDim.x) {
    int a = e / D, j = e % D;
    T mx = zerov<T>(), my = zerov<T>();
    if (j < Dk) {
      double sn = S.s[j] / c0, sq = sqrt(sn);
      mx = S.sa[a + j * FIT_RMAX] * (sq / S.s[j]);
      my = conjv(S.sv[a + j * FIT_RMAX]) * sq;
    }
    MXo[(size_t)it * R * D + e] = mx;
    MYo[(size_t)it * R * D + e] = my;
  }
  if (st && tid == 0) {
    st[2] = eps;
    st[3] = N > 0 ? eps / N : 0.0;
    st[5] = Dk;
    st[6] = iters;
    st[7] = n_eig;
    st[8] = isfinite(eps) && isfinite(N) ? 0.0 : 1.0;
    for (int j = 0; j < D; ++j) st[16 + 4 * fp.n_iter + j] = j < Dk ? S.s[j] / c0 : 0.0;
  }
}

hipError_t launch_bond_fit(bool cplx, int batch, int D, int R, const void* g, const void* RX, const void* RY,
                           const FitParams& fp, void* MX, void* MY, double* stats, int stats_stride, void* ws,
                           hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (R > FIT_RMAX || D > FIT_RMAX || R * D > 256) return hipErrorInvalidValue;
  size_t el = cplx ? 16 : 8;
  size_t shm = (size_t)(R * R + 7 * FIT_RMAX * FIT_RMAX) * el + (FIT_RMAX + 16 * 64 + 64) * 8 + FIT_RMAX * FIT_RMAX * 4;
  if (cplx)
    hipLaunchKernelGGL(k_bond_fit<cd>, dim3(batch), dim3(FIT_THREADS), shm, st, D, R, (const cd*)g, (const cd*)RX,
                       (const cd*)RY, fp, (cd*)MX, (cd*)MY, stats, stats_stride, (cd*)ws);
  else
    hipLaunchKernelGGL(k_bond_fit<double>, dim3(batch), dim3(FIT_THREADS), shm, st, D, R, (const double*)g,
                       (const double*)RX, (const double*)RY, fp, (double*)MX, (double*)MY, stats, stats_stride,
                       (double*)ws);
  return hipGetLastError();
}

}  // namespace ntu
