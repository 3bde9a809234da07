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
#include <algorithm>

namespace ntu {

constexpr int FIT_THREADS = 512;
constexpr int FIT_RMAX = 20;
// the group fit (k_bond_fit_grp)
constexpr int GRP_MAX = 16;                  // members per item
constexpr int GRP_CTL = 64;                  // control words per item (own cache lines):
                                             // [0] arrivals, [1] abort, [2] redo by k_bond_fit
constexpr unsigned GRP_SPIN_LIMIT = 1u << 20;
constexpr int GRP_NXMAX = 128;               // R Dn of the group path (R <= 16, Dn <= 8)
constexpr int GRP_MIN_D = 5;                 // smallest D the group path takes
static_assert(svdu_guess_elems() == 2 * FIT_RMAX * FIT_RMAX + 1, "guess layout");


// per-item global workspace (elements of T)
NTU_HD long long fit_ws_elems(int D, int R) {
  long long n = (long long)R * R, nx = (long long)R * D;
  return n * nx      // G1
         + 3 * nx * nx  // g_s, A (Cholesky / eigen), X (inverse / eigenvectors)
         + 3 * n;       // g y, d, g d
}

NTU_HD size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// the group fit's exchange area after the items' blocks: control words,
// [2][n] row values per item (by barrier parity), [2][GRP_MAX][2] partial sums
NTU_HD size_t grp_xch_bytes(size_t el, int batch, int R) {
  return align256((size_t)batch * GRP_CTL * 4) + align256((size_t)batch * 2 * R * R * el) +
         align256((size_t)batch * 2 * GRP_MAX * 2 * 8);
}

size_t fit_workspace_bytes(bool cplx, int batch, int D, int R) {
  const size_t el = cplx ? 16 : 8;
  return align256((size_t)batch * fit_ws_elems(D, R) * el) + grp_xch_bytes(el, batch, R) + 512;
}

// ---------------------------------------------------------------------------
// Certification of g (once per bond, in the fit kernel): a successful
// Cholesky factorisation of g - s I with s = 10 tol_max ||g||_F proves
// lambda_min(g) > s up to a backward error far below s.  Every half-step
// matrix g_s = K^H g K has K with orthonormal (or exactly zero) columns, so
// its eigenvalues lie in [lambda_min(g), lambda_max(g)] and no tolerance of
// the ladder removes any of them.
// ---------------------------------------------------------------------------
constexpr int CHOL_BS = 16;

// bytes of the fixed part of the fit kernel's dynamic shared memory
NTU_HD size_t fit_shared_fixed_bytes(size_t el, int R) {
  size_t b = (size_t)(R * R + 7 * FIT_RMAX * FIT_RMAX) * el + (FIT_RMAX + 16 * 64 + 64) * 8 + FIT_RMAX * FIT_RMAX * 4;
  return (b + 15) / 16 * 16;
}

// elements of the fit kernel's shared work region (after the fixed part)
NTU_HD size_t fit_work_elems(int R, int D) {
  const size_t cert_el = R * R <= 256 ? (size_t)R * R * CHOL_BS : 0;
  const size_t solve_el = (size_t)R * D * CHOL_BS + CHOL_BS * CHOL_BS + 200 + 3 * 200;
  return cert_el > solve_el ? cert_el : solve_el;
}
// Real fits with R Dn <= FIT_PACKED_NX keep the ladder's eigenproblem in
// shared memory, packed (n (n + 1) / 2 doubles after the work region).
constexpr int FIT_PACKED_NX = 128;
NTU_HD size_t fit_packed_bytes(bool cplx, int R, int D) {
  const int nx = R * D;
  return (!cplx && nx <= FIT_PACKED_NX) ? ((size_t)nx * (nx + 1) / 2 * 8 + 15) / 16 * 16 : 0;
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

// out = g v for a Hermitian n x n g (row-major):
//   out[r] = sum_c conj(g[c][r]) v[c].
// Work item (r, part), r fastest, sums a contiguous range of c, so a wave
// reads consecutive entries of each row of g; the parts meet in mv
// (max(n, blockDim.x) elements of shared memory).  Whole block.
template <class T>
NTU_DEV void fit_matvec(const T* __restrict__ g, int n, const T* v, T* out, T* mv) {
  const int tid = threadIdx.x, parts = max(1, (int)blockDim.x / n), cs = (n + parts - 1) / parts;
  for (int wi = tid; wi < parts * n; wi += blockDim.x) {
    const int r = wi % n, part = wi / n;
    const int c1 = min(n, (part + 1) * cs);
    T acc = zerov<T>();
    for (int c0 = part * cs; c0 < c1; c0 += 8) {
      T gv[8];
#pragma unroll
      for (int l = 0; l < 8; ++l) gv[l] = c0 + l < c1 ? g[(size_t)(c0 + l) * n + r] : zerov<T>();
#pragma unroll
      for (int l = 0; l < 8; ++l)
        if (c0 + l < c1) acc += cmul(gv[l], v[c0 + l]);
    }
    mv[wi] = acc;
  }
  __syncthreads();
  for (int r = tid; r < n; r += blockDim.x) {
    T acc = zerov<T>();
    for (int part = 0; part < parts; ++part) acc += mv[part * n + r];
    out[r] = acc;
  }
  __syncthreads();
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
  fit_matvec<T>(g, n, d, gd, S.sa);
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
    scale = fmax(scale, sqrt(lanes32_sum(v)));
  }
  for (int j = 0; j < Dn; ++j) {
    T v = lane < R ? M[lane * FIT_RMAX + j] : zerov<T>();
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        T qi = lane < R ? Q[lane * FIT_RMAX + i] : zerov<T>();
        T h = lanes32_sum(cmul(qi, v));
        v -= qi * h;
      }
    double nn = sqrt(lanes32_sum(abs2(v)));
    double inv = (scale > 0 && nn > kappa * scale) ? 1.0 / nn : 0.0;
    if (lane < R) Q[lane * FIT_RMAX + j] = v * inv;
  }
}

// The same orthonormal basis for R <= 16 and Dn <= 8 with classical
// Gram-Schmidt applied twice.  A lane holds one row of every column (the four
// 16-lane rows of the wave hold the same matrix); in each projection pass the
// lanes of row g of the wave take the earlier columns g and g + 4 (row sums
// over 16 lanes), and the four rows' corrections meet by two lane exchanges,
// added in an order under which every row of the wave gets the same bits.
// Wave 0.
template <class T>
NTU_DEV T lane_xor_t(T v, int m);
template <> NTU_DEV double lane_xor_t<double>(double v, int m) { return __shfl_xor(v, m, 64); }
template <> NTU_DEV cd lane_xor_t<cd>(cd v, int m) { return cd{__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64)}; }
template <class T>
NTU_DEV T row_sum16_t(T v);
template <> NTU_DEV double row_sum16_t<double>(double v) { return row_sum16(v); }
template <> NTU_DEV cd row_sum16_t<cd>(cd v) { return cd{row_sum16(v.x), row_sum16(v.y)}; }

template <class T>
NTU_DEV void fit_orthonormalise16(const T* M, T* Q, int R, int Dn, double kappa) {
  if (threadIdx.x >= 64) return;
  const int row = threadIdx.x & 15, g = (threadIdx.x >> 4) & 3;
  T q[8];
  double scale = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const T v = (j < Dn && row < R) ? M[row * FIT_RMAX + j] : zerov<T>();
    q[j] = v;  // the columns of M for now
    scale = fmax(scale, sqrt(row_sum16(abs2(v))));
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (j >= Dn) break;
    // this row's two earlier columns
    const T qa = g == 0 ? q[0] : g == 1 ? q[1] : g == 2 ? q[2] : q[3];
    const T qb = g == 0 ? q[4] : g == 1 ? q[5] : g == 2 ? q[6] : q[7];
    const bool ua = g < j, ub = g + 4 < j;
    T v = q[j];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const T ha = row_sum16_t<T>(cmul(qa, v)), hb = row_sum16_t<T>(cmul(qb, v));
      T c = zerov<T>();
      if (ua) c += qa * ha;
      if (ub) c += qb * hb;
      c += lane_xor_t<T>(c, 16);
      c += lane_xor_t<T>(c, 32);
      v -= c;
    }
    const double nn = sqrt(row_sum16(abs2(v)));
    const double inv = (scale > 0 && nn > kappa * scale) ? 1.0 / nn : 0.0;
    q[j] = v * inv;
  }
  if (threadIdx.x < 16 && row < R)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < Dn) Q[row * FIT_RMAX + j] = q[j];
}

// Thin QR of the R x Dn matrix M (row-major, stride FIT_RMAX) by Gram-Schmidt
// with the projection applied twice: Q (R x Dn) and the upper triangular Rf
// (Dn x Dn, row-major, stride FIT_RMAX), M = Q Rf up to dropped residuals of
// dependent columns (norm <= kappa * largest column norm), whose Q column and
// diagonal entry are then exactly zero.  Wave `wv` of the block.
template <class T>
NTU_DEV void fit_qr_small(const T* M, T* Q, T* Rf, int R, int Dn, double kappa, int wv) {
  if ((int)(threadIdx.x >> 6) != wv) return;
  const int lane = threadIdx.x & 63;
  double scale = 0;
  for (int j = 0; j < Dn; ++j) {
    double v = lane < R ? abs2(M[lane * FIT_RMAX + j]) : 0.0;
    scale = fmax(scale, sqrt(lanes32_sum(v)));
  }
  for (int e = lane; e < Dn * FIT_RMAX; e += 64) Rf[e] = zerov<T>();
  for (int j = 0; j < Dn; ++j) {
    T v = lane < R ? M[lane * FIT_RMAX + j] : zerov<T>();
    T racc = zerov<T>();  // lane i < j accumulates Rf[i][j]
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        T qi = lane < R ? Q[lane * FIT_RMAX + i] : zerov<T>();
        T h = lanes32_sum(cmul(qi, v));
        v -= qi * h;
        if (lane == i) racc += h;
      }
    double nn = sqrt(lanes32_sum(abs2(v)));
    const bool keep = scale > 0 && nn > kappa * scale;
    if (lane < R) Q[lane * FIT_RMAX + j] = v * (keep ? 1.0 / nn : 0.0);
    if (lane < j) Rf[lane * FIT_RMAX + j] = racc;
    if (lane == j) Rf[j * FIT_RMAX + j] = realv<T>(keep ? nn : 0.0);
  }
}

// Solve the half-step system gs m = J (see the file comment).  gs: nx x nx in
// global memory.  Returns the chosen tolerance; *used_eig = 1 if the ladder
// was evaluated through the eigendecomposition.  `eval(m)` must return the
// error of candidate m (whole-block call).
template <class T, class Eval>
NTU_DEV double fit_solve(const T* gs, int nx, const FitParams& fp, const FitShared<T>& S, T* A, T* X,
                         double N, int* used_eig, Eval eval, double* Ap) {
  __shared__ int m_sh, cnt, rcnt[2];
  __shared__ double pc[256], ps[256];
  __shared__ T pe[256];
  __shared__ int pq[256];
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
  bool packed = false;
  if constexpr (!is_cplx<T>::value) {
    if (Ap != nullptr && m <= FIT_PACKED_NX) {
      // real: the lower triangle in shared memory; the eigenvalues then go to
      // the diagonal of A, where the ladder below reads them
      packed = true;
      for (int e = tid; e < m * (m + 1) / 2; e += blockDim.x) {
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= e) ++i;
        while (i * (i + 1) / 2 > e) --i;
        const int j = e - i * (i + 1) / 2;
        Ap[e] = gs[(size_t)S.idx[i] * nx + S.idx[j]];
      }
      __syncthreads();
      block_jacobi_eigh_packed(Ap, m, X, m, pc, ps, pq, &cnt, rcnt, fro);
      for (int i = tid; i < m; i += blockDim.x) A[(size_t)i * m + i] = Ap[packed_at(i, i)];
      __syncthreads();
    }
  }
  if (!packed) {
    for (long long e = tid; e < (long long)m * m; e += blockDim.x)
      A[e] = gs[(size_t)S.idx[e / m] * nx + S.idx[e % m]];
    __syncthreads();
    block_jacobi_eigh<T>(A, m, m, X, m, pc, ps, pe, pq, &cnt, fro);
  }
  double lmax = -INFINITY;
  for (int i = tid; i < m; i += blockDim.x) lmax = fmax(lmax, rev(A[(size_t)i * m + i]));
  lmax = block_max(lmax, S.red);
  if (!(lmax > 0.0)) return tol_max;  // nothing positive to invert: m = 0
  // component r of eigenvector i (the packed solver stores them transposed)
  const size_t xr = packed ? 1 : (size_t)m, xi = packed ? (size_t)m : 1;
  __shared__ T proj[256];
  for (int i = tid; i < m; i += blockDim.x) {
    T acc = zerov<T>();
    for (int r = 0; r < m; ++r) acc += cmul(X[r * xr + i * xi], S.J[S.idx[r]]);
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
        if (l > thr) acc += X[r * xr + i * xi] * proj[i] * (1.0 / l);
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
      if (l > thr) acc += X[r * xr + i * xi] * proj[i] * (1.0 / l);
    }
    S.m[S.idx[r]] = acc;
  }
  __syncthreads();
  return fp.tol[best];
}


// ---------------------------------------------------------------------------
// Half-step matrix g_s = K^H g K and J = K^H g y in two block-wide passes
// (K = I (x) Q for the X half-step, parameters (a, j); K = Q (x) I for the
// Y half-step, parameters (j, b)):
//   pass 1  G1[r][(x, j)] = sum_y g[r][col(x, y)] Q[y][j]
//                         = sum_y conj(g[col(x, y)][r]) Q[y][j]   (g Hermitian)
//           X: col = x R + y, G1 column x Dn + j;  Y: col = y R + x, column j R + x
//   pass 2  g_s[(o, j')][c] = sum_i conj(Q[i][j']) G1[row(o, i)][c]
//           X: row = o R + i, g_s row o Dn + j';   Y: row = i R + o, row j' R + o
// Pass 1 runs r fastest (coalesced reads of g), pass 2 c fastest.  Each
// thread carries FORM_JB columns of Q in registers.
// ---------------------------------------------------------------------------
constexpr int FAST_NX = 200;        // largest R D on the certified path (R <= 20, D <= 10)
constexpr int FIT_CERT_NMAX = 256;  // largest R^2 certified by the shifted Cholesky
constexpr int FORM_JB = 8;          // columns of Q per thread
constexpr int FORM_LB = 8;          // loads issued together
constexpr int CG_NX = 200;          // largest R D solved by conjugate gradients

template <class T>
NTU_DEV void form_gs(const T* __restrict__ Gm, const T* __restrict__ gyv, int R, int Dn, int half, const T* Q,
                     T* __restrict__ G1, T* __restrict__ gs, T* J) {
  const int tid = threadIdx.x, nt = blockDim.x, n = R * R, nx = R * Dn;
  const int njb = (Dn + FORM_JB - 1) / FORM_JB;
  const int w1 = n * R * njb;
  for (int e = tid; e < w1; e += nt) {
    const int r = e % n, t = e / n, x = t % R, jb = t / R;
    T acc[FORM_JB];
#pragma unroll
    for (int u = 0; u < FORM_JB; ++u) acc[u] = zerov<T>();
    for (int y0 = 0; y0 < R; y0 += FORM_LB) {
      // FORM_LB loads in flight, then their products
      T gv[FORM_LB];
#pragma unroll
      for (int l = 0; l < FORM_LB; ++l) {
        const int y = y0 + l;
        const int col = half == 0 ? x * R + y : y * R + x;
        gv[l] = y < R ? conjv(Gm[(size_t)col * n + r]) : zerov<T>();
      }
#pragma unroll
      for (int l = 0; l < FORM_LB; ++l) {
        const T* qy = Q + min(y0 + l, R - 1) * FIT_RMAX + jb * FORM_JB;
#pragma unroll
        for (int u = 0; u < FORM_JB; ++u) acc[u] += gv[l] * qy[u];
      }
    }
#pragma unroll
    for (int u = 0; u < FORM_JB; ++u) {
      const int j = jb * FORM_JB + u;
      if (j < Dn) G1[(size_t)r * nx + (half == 0 ? x * Dn + j : j * R + x)] = acc[u];
    }
  }
  __syncthreads();
  const int w2 = nx * R * njb;
  for (int e = tid; e < w2; e += nt) {
    const int c = e % nx, t = e / nx, o = t % R, jb = t / R;
    T acc[FORM_JB];
#pragma unroll
    for (int u = 0; u < FORM_JB; ++u) acc[u] = zerov<T>();
    for (int i0 = 0; i0 < R; i0 += FORM_LB) {
      T v[FORM_LB];
#pragma unroll
      for (int l = 0; l < FORM_LB; ++l) {
        const int i = i0 + l;
        v[l] = i < R ? G1[(size_t)(half == 0 ? o * R + i : i * R + o) * nx + c] : zerov<T>();
      }
#pragma unroll
      for (int l = 0; l < FORM_LB; ++l) {
        const T* qi = Q + min(i0 + l, R - 1) * FIT_RMAX + jb * FORM_JB;
#pragma unroll
        for (int u = 0; u < FORM_JB; ++u) acc[u] += cmul(qi[u], v[l]);
      }
    }
#pragma unroll
    for (int u = 0; u < FORM_JB; ++u) {
      const int j = jb * FORM_JB + u;
      if (j < Dn) gs[(size_t)(half == 0 ? o * Dn + j : j * R + o) * nx + c] = acc[u];
    }
  }
  // J[(o, j')] = sum_i conj(Q[i][j']) gy[row(o, i)]
  for (int e = tid; e < nx; e += nt) {
    const int o = half == 0 ? e / Dn : e % R, jp = half == 0 ? e % Dn : e / R;
    T acc = zerov<T>();
    for (int i = 0; i < R; ++i) acc += cmul(Q[i * FIT_RMAX + jp], gyv[half == 0 ? o * R + i : i * R + o]);
    J[e] = acc;
  }
  __syncthreads();
}

// The same two passes on the FP64 matrix cores (v_mfma_f64_16x16x4: lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// D[l / 16 + 4 v][l % 16]).  Complex products use two real products into one
// accumulator: with B' = [Re Q | Im Q] and B'' = [-Im Q | Re Q] (columns
// 0-7 | 8-15), Re(A) B' + Im(A) B'' = [Re(A Q) | Im(A Q)]; pass 2 stacks the
// rows the same way.  Each wave takes whole 16 x 16 output tiles.  Needs
// R <= FIT_RMAX, Dn <= 8 (complex) or 16 (real).
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class T, int NKC, int RC>
NTU_DEV void form_gs_mfma_k(const T* __restrict__ Gm, const T* __restrict__ gyv, int Rarg, int Dn, int half,
                            const T* Q, T* __restrict__ G1, T* __restrict__ gs, T* J) {
  constexpr bool CPLX = is_cplx<T>::value;
  const int R = RC > 0 ? RC : Rarg;  // compile-time R where instantiated
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int n = R * R, nx = R * Dn;
  const int l16 = lane & 15, lk = lane >> 4;
  double* G1d = (double*)G1;
  double* gsd = (double*)gs;
  // pass 1 B operands for every K chunk: row y = 4 kc + lk, column l16
  double b1[NKC], b2[NKC];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
    const int y = 4 * kc + lk;
    double v1 = 0.0, v2 = 0.0;
    if (y < R) {
      if constexpr (CPLX) {
        const int j = l16 & 7;
        if (j < Dn) {
          const T q = Q[y * FIT_RMAX + j];
          v1 = l16 < 8 ? rev(q) : imv(q);
          v2 = l16 < 8 ? -imv(q) : rev(q);
        }
      } else {
        if (l16 < Dn) v1 = rev(Q[y * FIT_RMAX + l16]);
      }
    }
    b1[kc] = v1;
    b2[kc] = v2;
  }
  const int nrt = (n + 15) / 16, nu1 = R * nrt;
  // the operands of the wave's next unit are loaded while the current one
  // runs on the matrix cores
  auto load1 = [&](int u, T (&gv)[NKC]) {
    const int x = u / nrt, r = (u % nrt) * 16 + l16;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const int y = 4 * kc + lk;
      // branch-free: invalid entries load element 0; the mask and the
      // conjugation are applied at the use (work on a loaded register here
      // would wait for the load)
      const bool ok = y < R && r < n;
      gv[kc] = Gm[ok ? (size_t)(half == 0 ? x * R + y : y * R + x) * n + r : 0];
    }
  };
  T gnext[NKC];
  load1(min(w, nu1 - 1), gnext);
  for (int u = w; u < nu1; u += nw) {
    const int x = u / nrt, r0 = (u % nrt) * 16;
    T gv[NKC];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) gv[kc] = gnext[kc];
    load1(min(u + nw, nu1 - 1), gnext);  // unconditional: stays in flight
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const bool ok = 4 * kc + lk < R && r0 + l16 < n;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ok ? rev(gv[kc]) : 0.0, b1[kc], acc, 0, 0, 0);
      if constexpr (CPLX) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ok ? -imv(gv[kc]) : 0.0, b2[kc], acc, 0, 0, 0);
    }
    // lane holds rows r0 + lk + 4 v, column l16
    const int j = CPLX ? (l16 & 7) : l16, part = CPLX ? (l16 >> 3) : 0;
    if (j < Dn) {
      const int c = half == 0 ? x * Dn + j : j * R + x;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = r0 + lk + 4 * v;
        if (rr < n) G1d[((size_t)rr * nx + c) * (CPLX ? 2 : 1) + part] = acc[v];
      }
    }
  }
  __syncthreads();
  // pass 2: A operands (rows j' stacked re / im for complex) for every K chunk
  double a1[NKC], a2[NKC];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
    const int i = 4 * kc + lk;
    double v1 = 0.0, v2 = 0.0;
    if (i < R) {
      if constexpr (CPLX) {
        const int jp = l16 & 7;
        if (jp < Dn) {
          const T q = Q[i * FIT_RMAX + jp];
          // conj(Q) = Pr + i Pi with Pr = Re Q, Pi = -Im Q;  A' = [Pr; Pi], A'' = [-Pi; Pr]
          v1 = l16 < 8 ? rev(q) : -imv(q);
          v2 = l16 < 8 ? imv(q) : rev(q);
        }
      } else {
        if (l16 < Dn) v1 = rev(Q[i * FIT_RMAX + l16]);
      }
    }
    a1[kc] = v1;
    a2[kc] = v2;
  }
  const int nct = (nx + 15) / 16, nu2 = R * nct;
  auto load2 = [&](int u, T (&gv)[NKC]) {
    const int o = u / nct, c = (u % nct) * 16 + l16;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const int i = 4 * kc + lk;
      const bool ok = i < R && c < nx;
      gv[kc] = G1[ok ? (size_t)(half == 0 ? o * R + i : i * R + o) * nx + c : 0];
    }
  };
  load2(min(w, nu2 - 1), gnext);
  for (int u = w; u < nu2; u += nw) {
    const int o = u / nct, c = (u % nct) * 16 + l16;
    T gv[NKC];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) gv[kc] = gnext[kc];
    load2(min(u + nw, nu2 - 1), gnext);  // unconditional: stays in flight
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const bool ok = 4 * kc + lk < R && c < nx;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[kc], ok ? rev(gv[kc]) : 0.0, acc, 0, 0, 0);
      if constexpr (CPLX) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[kc], ok ? imv(gv[kc]) : 0.0, acc, 0, 0, 0);
    }
    if (c < nx) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i16 = lk + 4 * v;
        const int jp = CPLX ? (i16 & 7) : i16, part = CPLX ? (i16 >> 3) : 0;
        if (jp < Dn) {
          const int row = half == 0 ? o * Dn + jp : jp * R + o;
          gsd[((size_t)row * nx + c) * (CPLX ? 2 : 1) + part] = acc[v];
        }
      }
    }
  }
  // J[(o, j')] = sum_i conj(Q[i][j']) gy[row(o, i)]
  for (int e = threadIdx.x; e < nx; e += blockDim.x) {
    const int o = half == 0 ? e / Dn : e % R, jp = half == 0 ? e % Dn : e / R;
    T acc = zerov<T>();
    for (int i = 0; i < R; ++i) acc += cmul(Q[i * FIT_RMAX + jp], gyv[half == 0 ? o * R + i : i * R + o]);
    J[e] = acc;
  }
  __syncthreads();
}

// Kept out of line: the formation gets the kernel's full register budget
// for its loads in flight instead of sharing it with the rest of the fit.
template <class T>
__device__ __noinline__ void form_gs_mfma(const T* __restrict__ Gm, const T* __restrict__ gyv, int R, int Dn, int half, const T* Q,
                          T* __restrict__ G1, T* __restrict__ gs, T* J) {
  switch (R) {  // the enlarged bond dimensions of a rank-2 gate on the certified path
    case 4: form_gs_mfma_k<T, 1, 4>(Gm, gyv, R, Dn, half, Q, G1, gs, J); return;
    case 6: form_gs_mfma_k<T, 2, 6>(Gm, gyv, R, Dn, half, Q, G1, gs, J); return;
    case 8: form_gs_mfma_k<T, 2, 8>(Gm, gyv, R, Dn, half, Q, G1, gs, J); return;
    case 10: form_gs_mfma_k<T, 3, 10>(Gm, gyv, R, Dn, half, Q, G1, gs, J); return;
    case 12: form_gs_mfma_k<T, 3, 12>(Gm, gyv, R, Dn, half, Q, G1, gs, J); return;
    case 14: form_gs_mfma_k<T, 4, 14>(Gm, gyv, R, Dn, half, Q, G1, gs, J); return;
    case 16: form_gs_mfma_k<T, 4, 16>(Gm, gyv, R, Dn, half, Q, G1, gs, J); return;
    default: break;
  }
  switch ((R + 3) / 4) {
    case 1: form_gs_mfma_k<T, 1, 0>(Gm, gyv, R, Dn, half, Q, G1, gs, J); break;
    case 2: form_gs_mfma_k<T, 2, 0>(Gm, gyv, R, Dn, half, Q, G1, gs, J); break;
    case 3: form_gs_mfma_k<T, 3, 0>(Gm, gyv, R, Dn, half, Q, G1, gs, J); break;
    case 4: form_gs_mfma_k<T, 4, 0>(Gm, gyv, R, Dn, half, Q, G1, gs, J); break;
    default: form_gs_mfma_k<T, 5, 0>(Gm, gyv, R, Dn, half, Q, G1, gs, J); break;
  }
}

// Dependent directions (zero columns of Q) of g_s: unit rows and columns,
// zero right-hand side.  zcol[j] != 0 marks column j of Q.  Whole block.
template <class T>
NTU_DEV void deflate_gs(T* gs, T* J, int R, int Dn, int half, const int* zcol) {
  bool anyz = false;
  for (int j = 0; j < Dn; ++j) anyz = anyz || zcol[j] != 0;
  if (!anyz) return;
  const int nx = R * Dn;
  for (int e = threadIdx.x; e < nx * nx; e += blockDim.x) {
    const int i = e / nx, j = e % nx;
    const int ji = half == 0 ? i % Dn : i / R, jj = half == 0 ? j % Dn : j / R;
    if (zcol[ji] || zcol[jj]) gs[e] = realv<T>(i == j ? 1.0 : 0.0);
  }
  for (int e = threadIdx.x; e < nx; e += blockDim.x)
    if (zcol[half == 0 ? e % Dn : e / R]) J[e] = zerov<T>();
  __syncthreads();
}

template <class T>
NTU_DEV bool chol_certify(T* Wc, int n, T* pan, int* flag) {
  return blocked_cholesky<T, CHOL_BS>(Wc, n, n, pan, flag);
}

// Conjugate gradients for g_s m = J (g_s Hermitian positive definite, nx x nx
// in global memory, dependent directions already deflated), from m = 0 or,
// with warm, from the m given (the stopping rule stays relative to |J|).  The product
// q = g_s p reads g_s column-wise through its Hermitian symmetry, r fastest,
// with the partial sums meeting in mv (blockDim.x elements).  p, q, r: nx
// elements of shared memory.  Iterates to a relative residual of rtol (at
// most max_it iterations); returns false if it does not get there.
template <class T>
NTU_DEV bool cg_solve(const T* __restrict__ gs, int nx, const T* J, T* m, T* p, T* q, T* r, T* mv, double* red,
                      double rtol, int max_it, int* iters_out, bool warm) {
  const int tid = threadIdx.x, parts = (int)blockDim.x / nx, cs = (nx + parts - 1) / parts;
  // dst = g_s src, read column-wise through the Hermitian symmetry; the parts
  // meet in mv; ends with a barrier
  auto matvec = [&](const T* src, T* dst) {
    if (tid < parts * nx) {
      const int i = tid % nx, part = tid / nx;
      const int j1 = min(nx, (part + 1) * cs);
      T acc = zerov<T>();
      for (int j0 = part * cs; j0 < j1; j0 += FORM_LB) {
        T v[FORM_LB];
#pragma unroll
        for (int l = 0; l < FORM_LB; ++l) v[l] = j0 + l < j1 ? gs[(size_t)(j0 + l) * nx + i] : zerov<T>();
#pragma unroll
        for (int l = 0; l < FORM_LB; ++l)
          if (j0 + l < j1) acc += cmul(v[l], src[j0 + l]);
      }
      mv[tid] = acc;
    }
    __syncthreads();
    for (int e = tid; e < nx; e += blockDim.x) {
      T acc = zerov<T>();
      for (int part = 0; part < parts; ++part) acc += mv[part * nx + e];
      dst[e] = acc;
    }
    __syncthreads();
  };
  double bb = 0;
  for (int e = tid; e < nx; e += blockDim.x) {
    if (!warm) m[e] = zerov<T>();
    bb += abs2(J[e]);
  }
  bb = block_sum(bb, red);  // contains barriers: m visible
  // r = J - g_s m (m = 0 unless warm), p = r
  if (warm) matvec(m, q);
  double rr = 0;
  for (int e = tid; e < nx; e += blockDim.x) {
    const T v = warm ? J[e] - q[e] : J[e];
    r[e] = v;
    p[e] = v;
    rr += abs2(v);
  }
  rr = block_sum(rr, red);
  const double stop = rtol * rtol * bb;
  int it = 0;
  bool conv = rr <= stop;
  for (; it < max_it && !conv; ++it) {
    matvec(p, q);
    double pq = 0;
    for (int e = tid; e < nx; e += blockDim.x) pq += rev(cmul(p[e], q[e]));
    pq = block_sum(pq, red);
    if (!(pq > 0.0)) break;
    const double alpha = rr / pq;
    double rn = 0;
    for (int e = tid; e < nx; e += blockDim.x) {
      m[e] += alpha * p[e];
      r[e] -= alpha * q[e];
      rn += abs2(r[e]);
    }
    rn = block_sum(rn, red);
    const double beta = rn / rr;
    rr = rn;
    conv = rn <= stop;
    for (int e = tid; e < nx; e += blockDim.x) p[e] = r[e] + beta * p[e];
    __syncthreads();
  }
  *iters_out = it;
  return conv;
}

// Solve g_s m = J by a blocked Cholesky factorisation of g_s (in place in
// global memory).  Rows of dependent (zero) directions of Q are replaced by
// unit rows with zero right-hand side, which is the same as leaving them out.
// Returns false if the factorisation fails (the caller then takes the
// eigendecomposition path, which reassembles g_s).
template <class T>
NTU_DEV bool fast_solve(T* gs, int R, int Dn, int half, const T* Q, const FitShared<T>& S, T* pan, T* dblk,
                        T* bz, int* flag) {
  const int nx = R * Dn;
  __shared__ int zcol[FIT_RMAX];
  if (threadIdx.x < Dn) {
    bool z = true;
    for (int i = 0; i < R; ++i) z = z && rev(Q[i * FIT_RMAX + threadIdx.x]) == 0.0 && imv(Q[i * FIT_RMAX + threadIdx.x]) == 0.0;
    zcol[threadIdx.x] = z ? 1 : 0;
  }
  __syncthreads();
  bool anyz = false;
  for (int j = 0; j < Dn; ++j) anyz = anyz || zcol[j];
  if (anyz) {
    for (long long e = threadIdx.x; e < (long long)nx * nx; e += blockDim.x) {
      const int i = (int)(e / nx), j = (int)(e % nx);
      const int ji = half == 0 ? i % Dn : i / R, jj = half == 0 ? j % Dn : j / R;
      if (zcol[ji] || zcol[jj]) gs[e] = realv<T>(i == j ? 1.0 : 0.0);
    }
  }
  for (int e = threadIdx.x; e < nx; e += blockDim.x) {
    const int je = half == 0 ? e % Dn : e / R;
    bz[e] = zcol[je] ? zerov<T>() : S.J[e];
  }
  __syncthreads();
  if (!blocked_cholesky<T, CHOL_BS>(gs, nx, nx, pan, flag)) return false;
  blocked_chol_solve<T, CHOL_BS>(gs, nx, nx, bz, S.m, dblk);
  return true;
}

// Balance (Fig. 5(d)): SVD of MX MY^T, normalised by the largest singular
// value.  With MX = Qx Rx and MY = Qy Ry, MX MY^T = Qx (Rx Ry^T) Qy^T, so for
// Rx Ry^T = Uc S Vc^H the singular vectors are U = Qx Uc, V = conj(Qy) Vc:
// a Dn x Dn SVD instead of an R x R one.  Writes MX = U S^1/2, MY = conj(V)
// S^1/2 (R x D, zero beyond the kept Dk columns) to MXi, MYi and leaves the
// singular values in S.s.  Buffers: Qx -> Qf, Qy -> J, Rx -> sa, Ry -> sv,
// C = Rx Ry^T (column-major) -> m, each FIT_RMAX^2.  Whole block; returns Dk.
template <class T>
NTU_DEV int fit_balance(int D, int R, int Dn, double kappa, const FitShared<T>& S, T* MXi, T* MYi, int* flag) {
  const int tid = threadIdx.x;
  __syncthreads();
  if (Dn > 0) {
    fit_qr_small<T>(S.MX, S.Qf, S.sa, R, Dn, kappa, 0);
    fit_qr_small<T>(S.MY, S.J, S.sv, R, Dn, kappa, 1);
    __syncthreads();
    for (int e = tid; e < Dn * Dn; e += blockDim.x) {
      const int i = e % Dn, k = e / Dn;
      T v = zerov<T>();
      for (int l = (i > k ? i : k); l < Dn; ++l) v += S.sa[i * FIT_RMAX + l] * S.sv[k * FIT_RMAX + l];
      S.m[i + k * FIT_RMAX] = v;
    }
    __syncthreads();
    svd_block_small<T>(S.m, Dn, Dn, FIT_RMAX, S.sv, FIT_RMAX, S.s, flag);
  } else {
    if (tid == 0) S.s[0] = 0.0;
    __syncthreads();
  }
  const double c0 = S.s[0];
  int Dk = 0;
  if (c0 > 0)
    for (int j = 0; j < Dn && Dk < D; ++j)
      if (S.s[j] > kappa * c0) ++Dk;
  for (int e = tid; e < R * D; e += blockDim.x) {
    int a = e / D, j = e % D;
    T mx = zerov<T>(), my = zerov<T>();
    if (j < Dk) {
      double sn = S.s[j] / c0, sq = sqrt(sn);
      T us = zerov<T>(), vv = zerov<T>();
      for (int i = 0; i < Dn; ++i) {
        us += S.Qf[a * FIT_RMAX + i] * S.m[i + j * FIT_RMAX];          // (U S)[a][j]
        vv += conjv(S.J[a * FIT_RMAX + i]) * S.sv[i + j * FIT_RMAX];   // V[a][j]
      }
      mx = us * (sq / S.s[j]);
      my = conjv(vv) * sq;
    }
    MXi[e] = mx;
    MYi[e] = my;
  }
  return Dk;
}

// SVDU guess (Fig. 2(c,d)): P = RX RY^T = U S V^H (one-sided Jacobi),
// Dn = min(D, #{S_j > kappa S_0}), MX = U S^1/2, MY = conj(V) S^1/2, row-major
// R x FIT_RMAX and zero beyond column Dn.  Leaves vec(P) (row-major) in y;
// sa, sv (FIT_RMAX^2) and s (FIT_RMAX) are scratch.  Whole block; returns Dn.
template <class T>
NTU_DEV int svdu_guess_dev(int D, int R, const T* RXi, const T* RYi, double kappa, T* y, T* sa, T* sv, double* s,
                           T* MX, T* MY, int* flag) {
  const int tid = threadIdx.x, n = R * R;
  for (int e = tid; e < n; e += blockDim.x) {
    int a = e / R, b = e % R;
    T v = zerov<T>();
    for (int k = 0; k < R; ++k) v += RXi[a * R + k] * RYi[b * R + k];
    y[e] = v;
    sa[a + b * FIT_RMAX] = v;
  }
  __syncthreads();
  svd_block_small<T>(sa, R, R, FIT_RMAX, sv, FIT_RMAX, s, flag);
  const double s0 = s[0];
  int Dn = 0;
  if (s0 > 0)
    for (int j = 0; j < R && Dn < D; ++j)
      if (s[j] > kappa * s0) ++Dn;
  // columns of sa are U s
  for (int e = tid; e < R * FIT_RMAX; e += blockDim.x) {
    int a = e / FIT_RMAX, j = e % FIT_RMAX;
    T mx = zerov<T>(), my = zerov<T>();
    if (j < Dn) {
      double sq = sqrt(s[j]);
      mx = sa[a + j * FIT_RMAX] * (1.0 / sq);
      my = conjv(sv[a + j * FIT_RMAX]) * sq;
    }
    MX[e] = mx;
    MY[e] = my;
  }
  __syncthreads();
  return Dn;
}

// The SVDU guess of every item, for a fit launched later (one block per item).
// guess[item]: MX (FIT_RMAX^2 elements, row-major R x FIT_RMAX), MY (the
// same), then Dn as the real part of one element.
template <class T>
__global__ void __launch_bounds__(FIT_THREADS) k_svdu_guess(int D, int R, const T* __restrict__ RX,
                                                            const T* __restrict__ RY, double kappa, T* guess) {
  __shared__ T y[FIT_RMAX * FIT_RMAX], sa[FIT_RMAX * FIT_RMAX], sv[FIT_RMAX * FIT_RMAX];
  __shared__ T MX[FIT_RMAX * FIT_RMAX], MY[FIT_RMAX * FIT_RMAX];
  __shared__ double s[FIT_RMAX];
  __shared__ int flag;
  const int it = blockIdx.x, n = R * R;
  const int Dn = svdu_guess_dev<T>(D, R, RX + (size_t)it * n, RY + (size_t)it * n, kappa, y, sa, sv, s, MX, MY, &flag);
  T* gi = guess + (size_t)it * svdu_guess_elems();
  for (int e = threadIdx.x; e < R * FIT_RMAX; e += blockDim.x) {
    gi[e] = MX[e];
    gi[FIT_RMAX * FIT_RMAX + e] = MY[e];
  }
  if (threadIdx.x == 0) gi[2 * FIT_RMAX * FIT_RMAX] = realv<T>((double)Dn);
}

template <class T>
__global__ void __launch_bounds__(FIT_THREADS) k_bond_fit(int D, int R, const T* __restrict__ g,
                                                          const T* __restrict__ RX, const T* __restrict__ RY,
                                                          FitParams fp, T* MXo, T* MYo, double* stats,
                                                          int stats_stride, T* ws, const double* cert,
                                                          const T* __restrict__ guess, const unsigned* redo) {
  extern __shared__ double shmem[];
  __shared__ int flag;
  const int it = blockIdx.x, tid = threadIdx.x;
  // after the group fit: only the items it left (redo flag set)
  if (redo && redo[(size_t)it * GRP_CTL + 2] == 0u) return;
  const int n = R * R;
  // without a metric (g == NULL: the SVDU scheme) the fit returns the
  // balanced SVDU guess: no certificate, no error, no iterations
  const T* G = g ? g + (size_t)it * n * n : nullptr;
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
  // after the fixed part, one work region used in turn for: the Cholesky panel
  // of the certification, and the Cholesky panel / diagonal block /
  // right-hand side of the half-step solve followed by the CG vectors
  T* work = (T*)((char*)shmem + fit_shared_fixed_bytes(sizeof(T), R));
  double* packed_lds = fit_packed_bytes(is_cplx<T>::value, R, D) > 0
                           ? (double*)((char*)work + fit_work_elems(R, D) * sizeof(T))
                           : nullptr;
  T* pan = work;
  T* dblk = work + (size_t)R * D * CHOL_BS;
  T* sbz = dblk + CHOL_BS * CHOL_BS;
  T* cgp = sbz + FAST_NX;
  T* cgq = cgp + CG_NX;
  T* cgr = cgq + CG_NX;
  __shared__ int chol_flag;
  __shared__ int zcol_sh[FIT_RMAX];
  int cg_iters_total = 0, cg_solves = 0;
  // certification: Cholesky of g - s I (copy in the workspace)
  bool certified = false;
  const bool cert_fits = (long long)n * n <= (long long)n * R * D + 3LL * R * D * R * D;
  int cert_kind = 0;  // 1: Gershgorin discs, 2: shifted Cholesky, 3: by the metric repair
  if (!G) {
  } else if (cert) {
    // the metric repair already tested the same two certificates on this g
    certified = R * D <= FAST_NX && cert[it] > 0.5;
    if (certified) cert_kind = 3;
  } else {
    if (R * D <= FAST_NX) certified = gershgorin_certify<T>(G, n, 10.0 * fp.tol[fp.n_tol - 1], S.red);
    if (certified) cert_kind = 1;
  }
  if (G && !cert && !certified && n <= FIT_CERT_NMAX && R * D <= FAST_NX && cert_fits) {
    T* Wc = W;  // n^2 elements fit in G1 .. X (cert_fits)
    double fro = 0;
    for (long long e = tid; e < (long long)n * n; e += blockDim.x) fro += abs2(G[e]);
    fro = sqrt(block_sum(fro, S.red));
    const double shift = 10.0 * fp.tol[fp.n_tol - 1] * fro;
    for (long long e = tid; e < (long long)n * n; e += blockDim.x) {
      T v = G[e];
      if (e / n == e % n) v = v - realv<T>(shift);
      Wc[e] = v;
    }
    __syncthreads();
    certified = fro > 0 && chol_certify<T>(Wc, n, pan, &chol_flag);
    if (certified) cert_kind = 2;
  }
  double* st = stats ? stats + (size_t)it * stats_stride : nullptr;
  const double kappa = fp.kappa;
  // phase cycle counters (thread 0): setup, g_s formation, solve, error, balance
  long long tph0 = 0, tph1 = 0, tph2 = 0, tph3 = 0, tph4 = 0;
  long long t_mark = clock64();
  auto tick = [&](int ph) {
    long long t = clock64();
    const long long dt = t - t_mark;
    if (ph == 0) tph0 += dt;
    else if (ph == 1) tph1 += dt;
    else if (ph == 2) tph2 += dt;
    else if (ph == 3) tph3 += dt;
    else tph4 += dt;
    t_mark = t;
  };

  int Dn;
  if (guess) {
    // the SVDU guess was computed beforehand (k_svdu_guess): read it, form y
    const T* gi = guess + (size_t)it * svdu_guess_elems();
    for (int e = tid; e < R * FIT_RMAX; e += blockDim.x) {
      S.MX[e] = gi[e];
      S.MY[e] = gi[FIT_RMAX * FIT_RMAX + e];
    }
    // RX and RY staged in shared memory (sa, sv: FIT_RMAX^2 >= R^2 each)
    for (int e = tid; e < n; e += blockDim.x) {
      S.sa[e] = RX[(size_t)it * n + e];
      S.sv[e] = RY[(size_t)it * n + e];
    }
    __syncthreads();
    for (int e = tid; e < n; e += blockDim.x) {
      int a = e / R, b = e % R;
      T v = zerov<T>();
      for (int k = 0; k < R; ++k) v += S.sa[a * R + k] * S.sv[b * R + k];
      S.y[e] = v;
    }
    Dn = (int)rev(gi[2 * FIT_RMAX * FIT_RMAX]);
  } else {
    Dn = svdu_guess_dev<T>(D, R, RX + (size_t)it * n, RY + (size_t)it * n, kappa, S.y, S.sa, S.sv, S.s, S.MX, S.MY,
                           &flag);
  }
  // g y and N
  __syncthreads();
  double N = 0, eps = 0.0;
  if (G) {
    fit_matvec<T>(G, n, S.y, gy, S.sa);
    for (int r = tid; r < n; r += blockDim.x) N += rev(cmul(S.y[r], gy[r]));
    N = block_sum(N, S.red);
    eps = Dn > 0 ? fit_error<T>(G, R, Dn, S, dv, gd) : 0.0;
  }
  if (st && tid == 0) {
    const int len = fit_stats_len(fp.n_iter, D);
    for (int i = 0; i < len; ++i) st[i] = 0.0;
    st[0] = N; st[1] = eps; st[4] = Dn;
  }
  __syncthreads();
  int iters = 0, n_eig = 0;
  double prev = eps;
  tick(0);
  for (int iter = 0; iter < fp.n_iter && Dn > 0 && G; ++iter) {
    for (int half = 0; half < 2; ++half) {
      // fixed factor F (MY for the X half-step, MX for the Y half-step), made isometric
      const T* F = half == 0 ? S.MY : S.MX;
      fit_orthonormalise<T>(F, S.Qf, R, Dn, kappa);
      __syncthreads();
      const int nx = R * Dn;
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
      double tau = fp.tol[fp.n_tol - 1];
      bool fast_done = false, have_est = false;
      double eps_est = 0.0;
      if (certified) {
        if (Dn <= (is_cplx<T>::value ? 8 : 16)) form_gs_mfma<T>(G, gy, R, Dn, half, S.Qf, G1, gs, S.J);
        else form_gs<T>(G, gy, R, Dn, half, S.Qf, G1, gs, S.J);
        tick(1);
        if (tid < Dn) {
          bool z = true;
          for (int i = 0; i < R; ++i) z = z && rev(S.Qf[i * FIT_RMAX + tid]) == 0.0 && imv(S.Qf[i * FIT_RMAX + tid]) == 0.0;
          zcol_sh[tid] = z ? 1 : 0;
        }
        __syncthreads();
        deflate_gs<T>(gs, S.J, R, Dn, half, zcol_sh);
        int cgi = 0;
        if (nx <= CG_NX) {
          // warm start: the current pair in this half-step's parameters.  The
          // fixed factor lies in the span of Q, F = Q W with W = Q^H F, so
          // X half: MX F^T = (MX W^T) Q^T;  Y half: F MY^T = Q (W MY^T).
          const T* Fx = half == 0 ? S.MY : S.MX;
          const T* Fr = half == 0 ? S.MX : S.MY;
          for (int e = tid; e < Dn * Dn; e += blockDim.x) {
            const int j = e / Dn, k = e % Dn;
            T w = zerov<T>();
            for (int b = 0; b < R; ++b) w += cmul(S.Qf[b * FIT_RMAX + j], Fx[b * FIT_RMAX + k]);
            S.sv[j * FIT_RMAX + k] = w;
          }
          __syncthreads();
          for (int e = tid; e < nx; e += blockDim.x) {
            const int a = half == 0 ? e / Dn : e % R, j = half == 0 ? e % Dn : e / R;
            T v = zerov<T>();
            for (int k = 0; k < Dn; ++k) v += Fr[a * FIT_RMAX + k] * S.sv[j * FIT_RMAX + k];
            S.m[e] = v;
          }
          fast_done = cg_solve<T>(gs, nx, S.J, S.m, cgp, cgq, cgr, S.sa, S.red, 1e-14, 64, &cgi, true);
          cg_iters_total += cgi;
          cg_solves += 1;
          if (fast_done) {
            // eps = m^H g_s m - 2 Re(m^H J) + N = N - Re(m^H (J + r)) with the
            // residual r = J - g_s m of the solve
            double pj = 0.0;
            for (int e = tid; e < nx; e += blockDim.x) pj += rev(cmul(S.m[e], S.J[e] + cgr[e]));
            eps_est = N - block_sum(pj, S.red);
            have_est = true;
          }
        }
        if (!fast_done) fast_done = fast_solve<T>(gs, R, Dn, half, S.Qf, S, pan, dblk, sbz, &chol_flag);
        tick(2);
      }
      // G1[(a' b'), c] :  X half: c = (a, j): sum_b g[(a' b'), (a b)] Q[b, j]
      //                   Y half: c = (j, b): sum_a g[(a' b'), (a b)] Q[a, j]
      if (!fast_done) {
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
      tau = fit_solve<T>(gs, nx, fp, S, A, X, N, &used_eig, eval, packed_lds);
      }  // !fast_done
      if (!fast_done) tick(2);
      set_free(S.m);
      // the residual form loses about log10(N / eps) digits: above 1e-8 N it is
      // kept, below that the error is evaluated directly
      if (have_est && eps_est > 1e-8 * N) eps = eps_est;
      else eps = fit_error<T>(G, R, Dn, S, dv, gd);
      tick(3);
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
  const int Dk = fit_balance<T>(D, R, Dn, kappa, S, MXo + (size_t)it * R * D, MYo + (size_t)it * R * D, &flag);
  tick(4);
  if (st && tid == 0) {
    st[9] = (double)cert_kind;
    st[15] = cg_solves > 0 ? (double)cg_iters_total / cg_solves : 0.0;
    st[10] = (double)tph0; st[11] = (double)tph1; st[12] = (double)tph2;
    st[13] = (double)tph3; st[14] = (double)tph4;
    st[2] = eps;
    st[3] = N > 0 ? eps / N : 0.0;
    st[5] = Dk;
    st[6] = iters;
    st[7] = n_eig;
    st[8] = isfinite(eps) && isfinite(N) ? 0.0 : 1.0;
    for (int j = 0; j < D; ++j) st[16 + 4 * fp.n_iter + j] = j < Dk ? S.s[j] / S.s[0] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Group fit: the certified fit of one item spread over G workgroups, the
// item's group (2 <= G <= R).  Every member keeps the small state (M_X, M_Y,
// the isometric factor, vec(P), g vec(P), the conjugate-gradient vectors)
// itself and does the same arithmetic on it in the same order, so the
// members reach the same decisions without exchanging them.  Split between
// them: the rows of g in the products with g (g vec(P), g d), and the rows of
// each half-step matrix g_s, which a member forms from its slabs of g into
// its own shared memory and multiplies in every conjugate-gradient iteration.
// Between members pass only the rows of a product and partial sums, through
// a per-item exchange area, one group barrier per iteration.
// Items the group does not take (no certificate from the metric repair, an
// empty guess, a solve that does not converge, a wait that runs out) are
// flagged and redone whole by k_bond_fit, launched after this kernel.
// ---------------------------------------------------------------------------

// Exchanged values are written and read with agent-scope atomic accesses,
// each coherent across the chip on its own; a writer's stores complete (the
// wait in grp_sync) before its workgroup arrives at the counter, and a reader
// loads only after it has seen the counter reach the barrier.  So the group
// barrier needs no cache write-back or invalidation.
NTU_DEV void xput(double* p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
NTU_DEV double xget(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
NTU_DEV void xput(cd* p, cd v) {
  xput(&p->x, v.x);
  xput(&p->y, v.y);
}
NTU_DEV cd xget(const cd* p) { return cd{xget(&p->x), xget(&p->y)}; }

// Group barrier on the item's arrival counter (count: the barriers this
// member has passed).  Bounded: a wait that runs out, or an abort raised by
// another member, returns false in every thread.  Whole block.
NTU_DEV bool grp_sync(unsigned* ctl, int G, unsigned& count, int* ok_sh) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's exchange stores have completed
  __syncthreads();
  ++count;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctl, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = count * (unsigned)G;
    unsigned spins = 0;
    int ok = 1;
    while (__hip_atomic_load(ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > GRP_SPIN_LIMIT) {
        __hip_atomic_store(ctl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *ok_sh = ok;
  }
  __syncthreads();
  return *ok_sh != 0;
}

// out_k[r - r0] = (g v_k)_r (k < nv <= 2) for the rows r0 <= r < r1 of a
// Hermitian n x n g, read column-wise: (g v)_r = sum_c conj(g[c][r]) v[c]
// with r fastest.  Work item (r, part); the parts meet in mv (blockDim.x
// elements per vector).  Whole block.
template <class T>
NTU_DEV void rows_matvec(const T* __restrict__ g, int n, int r0, int r1, int nv, const T* v0, const T* v1, T* o0,
                         T* o1, T* mv) {
  const int tid = threadIdx.x, nr = r1 - r0;
  const int parts = max(1, (int)blockDim.x / max(nr, 1)), cs = (n + parts - 1) / parts;
  if (tid < parts * nr) {
    const int r = r0 + tid % nr, part = tid / nr;
    const int c1 = min(n, (part + 1) * cs);
    T a0 = zerov<T>(), a1 = zerov<T>();
    for (int c0 = part * cs; c0 < c1; c0 += 8) {
      T gv[8];
#pragma unroll
      for (int l = 0; l < 8; ++l) gv[l] = c0 + l < c1 ? g[(size_t)(c0 + l) * n + r] : zerov<T>();
#pragma unroll
      for (int l = 0; l < 8; ++l)
        if (c0 + l < c1) {
          a0 += cmul(gv[l], v0[c0 + l]);
          if (nv > 1) a1 += cmul(gv[l], v1[c0 + l]);
        }
    }
    mv[tid] = a0;
    if (nv > 1) mv[blockDim.x + tid] = a1;
  }
  __syncthreads();
  for (int r = tid; r < nr; r += blockDim.x) {
    T s0 = zerov<T>(), s1 = zerov<T>();
    for (int part = 0; part < parts; ++part) {
      s0 += mv[part * nr + r];
      if (nv > 1) s1 += mv[blockDim.x + part * nr + r];
    }
    o0[r] = s0;
    if (nv > 1) o1[r] = s1;
  }
  __syncthreads();
}

// Rows of a half-step matrix from this member's slabs, on the FP64 matrix
// cores (v_mfma_f64_16x16x4: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]
// and receives D[l / 16 + 4 v][l % 16]).
//   X half: g_s[(a',j'),(a,j)] = sum_{b',b} conj(Q[b',j']) g[(a' b'),(a b)] Q[b,j],
//           rows (a', j') for the slabs a' = s0 .. s0 + nsl - 1, columns a Dn + j;
//   Y half: g_s[(j',b'),(j,b)] = sum_{a',a} conj(Q[a',j']) g[(a' b'),(a b)] Q[a,j],
//           rows (j', b') for the slabs b', columns j R + b.
// h holds the entries with the slab index leading in the contracted pair:
// h[(x R + y) ld + (x' - xoff) R + y'] = conj(entry of block (x', x) at
// (y', y)), i.e. g itself for the X half (ld = n, xoff = 0: its Hermitian
// symmetry gives lanes along the contiguous index) and the member's copy of
// the Y half's entries (k_bond_fit_grp).  A unit is one block (x', x): pass 1
// multiplies it by Q (complex as two real products into one accumulator,
// columns [Re | Im]), pass 2 by Q^H straight from the accumulator (register v
// of lane l is the B operand of K chunk v), and the real and imaginary parts
// are recombined across the two column halves of each 16-lane row (DPP
// rotate by 8).  Output: local row (x' - s0) Dn + j' of gsl (leading
// dimension gld).  Needs R <= 16, Dn <= 8.  Whole block.
template <class T, int NKC>
NTU_DEV void form_rows_mfma(const T* __restrict__ h, long long ld, int xoff, int R, int Dn, int half, int s0, int nsl,
                            const T* Q, T* gsl, int gld) {
  constexpr bool CPLX = is_cplx<T>::value;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  double b1[NKC], b2[NKC], a2[NKC];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
    const int y = 4 * kc + lk;
    double v1 = 0.0, v2 = 0.0, v3 = 0.0;
    if (y < R) {
      if constexpr (CPLX) {
        const int j = l16 & 7;
        if (j < Dn) {
          const T q = Q[y * FIT_RMAX + j];
          v1 = l16 < 8 ? rev(q) : imv(q);   // B' = [Re Q | Im Q]
          v2 = l16 < 8 ? -imv(q) : rev(q);  // B'' = [-Im Q | Re Q]
          v3 = l16 < 8 ? rev(q) : imv(q);   // pass 2: A = [Re Q^T ; Im Q^T]
        }
      } else {
        if (l16 < Dn) v1 = v3 = rev(Q[y * FIT_RMAX + l16]);
      }
    }
    b1[kc] = v1;
    b2[kc] = v2;
    a2[kc] = v3;
  }
  const int nu = nsl * R;
  // operands of unit u (clamped to the last unit, so that every load is
  // unconditional and the loads of the next units stay in flight while the
  // current ones are multiplied)
  auto load = [&](int u, T (&gv)[NKC]) {
    u = min(u, nu - 1);
    const int xl = u / R, x = u % R;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const int y = 4 * kc + lk;
      const bool ok = y < R && l16 < R;
      // raw: the mask and the conjugation are applied where the value is
      // used (work on a loaded register here would wait for the load)
      gv[kc] = h[ok ? (size_t)(x * R + y) * ld + (size_t)(s0 + xl - xoff) * R + l16 : 0];
    }
  };
  double* gd = (double*)gsl;
  auto unit = [&](int u, const T (&gv)[NKC]) {
    const int xl = u / R, x = u % R;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const bool ok = 4 * kc + lk < R && l16 < R;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ok ? rev(gv[kc]) : 0.0, b1[kc], acc, 0, 0, 0);
      if constexpr (CPLX) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ok ? -imv(gv[kc]) : 0.0, b2[kc], acc, 0, 0, 0);
    }
    f64x4 out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) out = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[kc], acc[kc], out, 0, 0, 0);
    if constexpr (CPLX) {
      // out rows 0-7: Re Q^T (G Q), rows 8-15: Im Q^T (G Q), columns [Re | Im];
      // g_s = Q^H G Q:  Re = out[j'][j] + out[8+j'][8+j],  Im = out[j'][8+j] - out[8+j'][j]
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const double t = dpp_move<0x128>(out[v + 2]);
        const double val = l16 < 8 ? out[v] + t : out[v] - t;
        const int jp = lk + 4 * v, j = l16 & 7, part = l16 >> 3;
        if (jp < Dn && j < Dn) {
          const int col = half == 0 ? x * Dn + j : j * R + x;
          gd[((size_t)(xl * Dn + jp) * gld + col) * 2 + part] = val;
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jp = lk + 4 * v, j = l16;
        if (jp < Dn && j < Dn) {
          const int col = half == 0 ? x * Dn + j : j * R + x;
          gd[(size_t)(xl * Dn + jp) * gld + col] = out[v];
        }
      }
    }
  };
  // two units per step, the next two in flight
  T ga[2][NKC], gb[2][NKC];
  load(w, ga[0]);
  load(w + nw, ga[1]);
  for (int u = w; u < nu; u += 2 * nw) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc) gb[p][kc] = ga[p][kc];
    load(u + 2 * nw, ga[0]);
    load(u + 3 * nw, ga[1]);
    unit(u, gb[0]);
    if (u + nw < nu) unit(u + nw, gb[1]);
  }
  __syncthreads();
}

template <class T>
__device__ __noinline__ void form_rows(const T* __restrict__ h, long long ld, int xoff, int R, int Dn, int half,
                                       int s0, int nsl, const T* Q, T* gsl, int gld) {
  switch ((R + 3) / 4) {
    case 1: form_rows_mfma<T, 1>(h, ld, xoff, R, Dn, half, s0, nsl, Q, gsl, gld); break;
    case 2: form_rows_mfma<T, 2>(h, ld, xoff, R, Dn, half, s0, nsl, Q, gsl, gld); break;
    case 3: form_rows_mfma<T, 3>(h, ld, xoff, R, Dn, half, s0, nsl, Q, gsl, gld); break;
    default: form_rows_mfma<T, 4>(h, ld, xoff, R, Dn, half, s0, nsl, Q, gsl, gld); break;
  }
}

// bytes of the group kernel's dynamic shared memory
NTU_HD size_t grp_gsl_elems(int R, int D, int G) {
  size_t gs = (size_t)((R + G - 1) / G) * D * (R * D + 1);
  return gs < 4 * FIT_RMAX * FIT_RMAX ? 4 * FIT_RMAX * FIT_RMAX : gs;  // the balancing's buffers alias it
}
NTU_HD size_t grp_shared_bytes(size_t el, int R, int D, int G) {
  const size_t n = (size_t)R * R;
  const size_t t_elems = 3 * 16 * FIT_RMAX + 3 * n + 7 * GRP_NXMAX + 8 * FIT_RMAX + 2 * FIT_THREADS + grp_gsl_elems(R, D, G);
  const size_t d_elems = 16 * 64 + FIT_RMAX + 64;
  return (t_elems * el + d_elems * 8 + 15) / 16 * 16;
}

template <class T>
__global__ void __launch_bounds__(FIT_THREADS) k_bond_fit_grp(int batch, int G, int D, int R, const T* __restrict__ g,
                                                              const T* __restrict__ RX, const T* __restrict__ RY,
                                                              FitParams fp, T* MXo, T* MYo, double* stats,
                                                              int stats_stride, T* ws, unsigned* ctl_all, T* xv_all,
                                                              double* xs_all, const double* cert,
                                                              const T* __restrict__ guess) {
  extern __shared__ double shmem[];
  __shared__ int sync_ok, flag;
  __shared__ int zcol_sh[FIT_RMAX];
  // workgroups are dealt to the eight XCDs in turn: the members of an item
  // take consecutive turns on one XCD
  const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
  const int it = (slot / G) * 8 + xcd, mem = slot % G;
  if (it >= batch) return;
  const int tid = threadIdx.x, n = R * R;
  const bool lead = mem == 0;
  unsigned* ctl = ctl_all + (size_t)it * GRP_CTL;
  T* xv = xv_all + (size_t)it * 2 * n;
  double* xs = xs_all + (size_t)it * 2 * GRP_MAX * 2;
  unsigned nsync = 0;
  auto redo = [&]() {
    if (lead && tid == 0) __hip_atomic_store(ctl + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  const T* G_ = g + (size_t)it * n * n;
  const T* gi = guess + (size_t)it * svdu_guess_elems();
  const int Dn = (int)rev(gi[2 * FIT_RMAX * FIT_RMAX]);
  if (!(R * D <= GRP_NXMAX && R <= 16 && D <= 8 && cert[it] > 0.5) || Dn < 1) {
    redo();
    return;
  }
  // this member's slabs (of the first index for the X half, of the second
  // for the Y half) and rows of g
  const int s0 = (mem * R) / G, s1 = ((mem + 1) * R) / G, nsl = s1 - s0;
  const int r0 = (mem * n) / G, r1 = ((mem + 1) * n) / G, nr = r1 - r0;
  // shared carve-up
  T* tp = (T*)shmem;
  T* MXs = tp; tp += 16 * FIT_RMAX;
  T* MYs = tp; tp += 16 * FIT_RMAX;
  T* Qf = tp; tp += 16 * FIT_RMAX;
  T* y = tp; tp += n;
  T* gy = tp; tp += n;
  T* dv = tp; tp += n;
  T* J = tp; tp += GRP_NXMAX;
  T* m = tp; tp += GRP_NXMAX;
  T* rv = tp; tp += GRP_NXMAX;
  T* pv = tp; tp += GRP_NXMAX;
  T* qv = tp; tp += GRP_NXMAX;
  T* o0 = tp; tp += GRP_NXMAX;   // this member's rows of a product with g (nr <= n / 2 <= 128)
  T* o1 = tp; tp += GRP_NXMAX;
  T* wsm = tp; tp += 8 * FIT_RMAX;
  T* mv = tp; tp += 2 * FIT_THREADS;
  T* gsl = tp; tp += grp_gsl_elems(R, D, G);
  const int gld = R * D + 1;
  double* red = (double*)tp;
  double* sv_s = red + 16 * 64;
  double* vec = sv_s + FIT_RMAX;
  double* st = (stats && lead) ? stats + (size_t)it * stats_stride : nullptr;
  long long tph0 = 0, tph1 = 0, tph2 = 0, tph3 = 0, tph4 = 0;
  long long t_mark = clock64();
  auto tick = [&](int ph) {
    const long long t = clock64(), dt = t - t_mark;
    if (ph == 0) tph0 += dt;
    else if (ph == 1) tph1 += dt;
    else if (ph == 2) tph2 += dt;
    else if (ph == 3) tph3 += dt;
    else tph4 += dt;
    t_mark = t;
  };
  // the guess (k_svdu_guess) and vec(P), in every member
  for (int e = tid; e < 16 * FIT_RMAX; e += blockDim.x) {
    MXs[e] = e < R * FIT_RMAX ? gi[e] : zerov<T>();
    MYs[e] = e < R * FIT_RMAX ? gi[FIT_RMAX * FIT_RMAX + e] : zerov<T>();
  }
  // vec(P) = vec(RX RY^T), RX and RY staged in shared memory first
  for (int e = tid; e < n; e += blockDim.x) {
    mv[e] = RX[(size_t)it * n + e];
    mv[n + e] = RY[(size_t)it * n + e];
  }
  __syncthreads();
  for (int e = tid; e < n; e += blockDim.x) {
    const int a = e / R, b = e % R;
    T v = zerov<T>();
    for (int k = 0; k < R; ++k) v += mv[a * R + k] * mv[n + b * R + k];
    y[e] = v;
  }
  // this member's copy of the Y half's entries (form_rows):
  // h[(x R + y) W + xl R + y'] = g[(y R + x), (y' R + s0 + xl)], W = nsl R
  T* hY = ws + (size_t)it * fit_ws_elems(D, R) + (size_t)n * R * s0;
  const int W = nsl * R;
  {
    // element f = (row R + y') nsl + xl: consecutive lanes read consecutive
    // entries of g; eight loads in flight per thread
    const int total = n * W;
    for (int f0 = tid; f0 < total; f0 += 8 * blockDim.x) {
      T v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int f = min(f0 + k * (int)blockDim.x, total - 1);
        const int xl = f % nsl, t = f / nsl, yp = t % R, row = t / R;
        v[k] = G_[(size_t)((row % R) * R + row / R) * n + yp * R + s0 + xl];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int f = f0 + k * (int)blockDim.x;
        if (f < total) {
          const int xl = f % nsl, t = f / nsl, yp = t % R, row = t / R;
          hY[(size_t)row * W + xl * R + yp] = v[k];
        }
      }
    }
  }
  __syncthreads();
  // d = vec(MX MY^T) - y
  auto form_d = [&]() {
    for (int e = tid; e < n; e += blockDim.x) {
      const int a = e / R, b = e % R;
      T v = zerov<T>();
      for (int j = 0; j < Dn; ++j) v += MXs[a * FIT_RMAX + j] * MYs[b * FIT_RMAX + j];
      dv[e] = v - y[e];
    }
    __syncthreads();
  };
  // partial sums of this member (k < 2) to the others; the group's sums in
  // member order
  auto exchange_sums = [&](double p0, double p1, double& t0, double& t1) -> bool {
    const int par = (nsync + 1) & 1;
    if (tid == 0) {
      xput(xs + (par * GRP_MAX + mem) * 2, p0);
      xput(xs + (par * GRP_MAX + mem) * 2 + 1, p1);
    }
    if (!grp_sync(ctl, G, nsync, &sync_ok)) return false;
    t0 = t1 = 0.0;
    for (int k = 0; k < G; ++k) {
      t0 += xget(xs + (par * GRP_MAX + k) * 2);
      t1 += xget(xs + (par * GRP_MAX + k) * 2 + 1);
    }
    return true;
  };
  // eps = d^H g d over the group
  auto group_error = [&](double& eps_out) -> bool {
    form_d();
    rows_matvec<T>(G_, n, r0, r1, 1, dv, nullptr, o0, nullptr, mv);
    double pe = 0.0;
    for (int r = tid; r < nr; r += blockDim.x) pe += rev(cmul(dv[r0 + r], o0[r]));
    pe = block_sum(pe, red);
    double dummy;
    return exchange_sums(pe, 0.0, eps_out, dummy);
  };
  // g y (rows exchanged), N = y^H g y and the guess's error d^H g d
  double N = 0.0, eps = 0.0;
  form_d();
  rows_matvec<T>(G_, n, r0, r1, 2, y, dv, o0, o1, mv);
  {
    double pn = 0.0, pe = 0.0;
    for (int r = tid; r < nr; r += blockDim.x) {
      pn += rev(cmul(y[r0 + r], o0[r]));
      pe += rev(cmul(dv[r0 + r], o1[r]));
      xput(xv + ((nsync + 1) & 1) * n + r0 + r, o0[r]);
    }
    pn = block_sum(pn, red);
    pe = block_sum(pe, red);
    if (!exchange_sums(pn, pe, N, eps)) {
      redo();
      return;
    }
    for (int e = tid; e < n; e += blockDim.x) gy[e] = xget(xv + (nsync & 1) * n + e);
    __syncthreads();
  }
  if (st && tid == 0) {
    const int len = fit_stats_len(fp.n_iter, D);
    for (int i = 0; i < len; ++i) st[i] = 0.0;
    st[0] = N; st[1] = eps; st[4] = Dn;
  }
  // q = g_s src over the group: this member's rows from gsl, exchanged
  int half = 0, nx = R * Dn;
  auto grow = [&](int l) { return half == 0 ? s0 * Dn + l : (l % Dn) * R + s0 + l / Dn; };
  // src in shared memory (visible to the whole block); the product q = g_s src
  // goes to every wave's registers, elements lane and lane + 64 (q0, q1)
  const int lane = tid & 63;
  auto group_matvec = [&](const T* src, T& q0, T& q1) -> bool {
    const int nrow = nsl * Dn, par = (nsync + 1) & 1;
    if (nrow * 16 <= (int)blockDim.x) {
      // 16 consecutive lanes per row, their partial sums added by DPP
      const int l = min(tid >> 4, nrow - 1), part = tid & 15;
      const T* row = gsl + (size_t)l * gld;
      T acc = zerov<T>();
      for (int c = part; c < nx; c += 16) acc += row[c] * src[c];
      if constexpr (is_cplx<T>::value) acc = T{row_sum16(acc.x), row_sum16(acc.y)};
      else acc = row_sum16(acc);
      if (part == 0 && (tid >> 4) < nrow) xput(xv + par * n + grow(l), acc);
    } else {
      const int parts = max(1, (int)blockDim.x / nrow);
      if (tid < parts * nrow) {
        const int l = tid % nrow, part = tid / nrow;
        const T* row = gsl + (size_t)l * gld;
        T acc = zerov<T>();
        for (int c = part; c < nx; c += parts) acc += row[c] * src[c];
        mv[tid] = acc;
      }
      __syncthreads();
      for (int l = tid; l < nrow; l += blockDim.x) {
        T acc = zerov<T>();
        for (int part = 0; part < parts; ++part) acc += mv[part * nrow + l];
        xput(xv + par * n + grow(l), acc);
      }
    }
    if (!grp_sync(ctl, G, nsync, &sync_ok)) return false;
    q0 = lane < nx ? xget(xv + par * n + lane) : zerov<T>();
    q1 = lane + 64 < nx ? xget(xv + par * n + lane + 64) : zerov<T>();
    return true;
  };
  int iters = 0, cg_iters_total = 0, cg_solves = 0;
  double prev = eps;
  const double tau = fp.tol[fp.n_tol - 1];
  const double kappa = fp.kappa;
  tick(0);
  bool ok = true;
  for (int iter = 0; iter < fp.n_iter && ok; ++iter) {
    for (half = 0; half < 2 && ok; ++half) {
      nx = R * Dn;
      const T* F = half == 0 ? MYs : MXs;
      fit_orthonormalise16<T>(F, Qf, R, Dn, kappa);
      __syncthreads();
      if (tid < Dn) {
        bool z = true;
        for (int i = 0; i < R; ++i) z = z && rev(Qf[i * FIT_RMAX + tid]) == 0.0 && imv(Qf[i * FIT_RMAX + tid]) == 0.0;
        zcol_sh[tid] = z ? 1 : 0;
      }
      // J[(o, j')] = sum_i conj(Q[i][j']) gy[row(o, i)]  (every member, all of it)
      for (int e = tid; e < nx; e += blockDim.x) {
        const int o = half == 0 ? e / Dn : e % R, jp = half == 0 ? e % Dn : e / R;
        T acc = zerov<T>();
        for (int i = 0; i < R; ++i) acc += cmul(Qf[i * FIT_RMAX + jp], gy[half == 0 ? o * R + i : i * R + o]);
        J[e] = acc;
      }
      if (lead) tick(0);
      if (half == 0) form_rows<T>(G_, n, 0, R, Dn, 0, s0, nsl, Qf, gsl, gld);
      else form_rows<T>(hY, W, s0, R, Dn, 1, s0, nsl, Qf, gsl, gld);
      // dependent directions (zero columns of Q): unit rows and columns, zero right-hand side
      bool anyz = false;
      for (int j = 0; j < Dn; ++j) anyz = anyz || zcol_sh[j] != 0;
      if (anyz) {
        const int nrow = nsl * Dn;
        for (int e = tid; e < nrow * nx; e += blockDim.x) {
          const int l = e / nx, c = e % nx, i = grow(l);
          const int ji = half == 0 ? i % Dn : i / R, jj = half == 0 ? c % Dn : c / R;
          if (zcol_sh[ji] || zcol_sh[jj]) gsl[(size_t)l * gld + c] = realv<T>(i == c ? 1.0 : 0.0);
        }
        for (int e = tid; e < nx; e += blockDim.x)
          if (zcol_sh[half == 0 ? e % Dn : e / R]) J[e] = zerov<T>();
      }
      if (lead) tick(1);
      // warm start: the current pair in this half-step's parameters (the
      // fixed factor lies in the span of Q: F = Q W with W = Q^H F)
      const T* Fx = half == 0 ? MYs : MXs;
      const T* Fr = half == 0 ? MXs : MYs;
      for (int e = tid; e < Dn * Dn; e += blockDim.x) {
        const int j = e / Dn, k = e % Dn;
        T wv = zerov<T>();
        for (int b = 0; b < R; ++b) wv += cmul(Qf[b * FIT_RMAX + j], Fx[b * FIT_RMAX + k]);
        wsm[j * FIT_RMAX + k] = wv;
      }
      __syncthreads();
      for (int e = tid; e < nx; e += blockDim.x) {
        const int a = half == 0 ? e / Dn : e % R, j = half == 0 ? e % Dn : e / R;
        T v = zerov<T>();
        for (int k = 0; k < Dn; ++k) v += Fr[a * FIT_RMAX + k] * wsm[j * FIT_RMAX + k];
        m[e] = v;
      }
      __syncthreads();
      if (lead) tick(0);
      // conjugate gradients (g_s certified positive definite).  Every member
      // holds every vector, and within a member every wave holds all of each
      // in registers (elements lane and lane + 64), so a dot product is one
      // wave sum, bit-identical in all waves and members; the product with
      // g_s is split over the group.  pv in shared memory feeds the product.
      const bool v0 = lane < nx, v1 = lane + 64 < nx;
      const T J0 = v0 ? J[lane] : zerov<T>(), J1 = v1 ? J[lane + 64] : zerov<T>();
      T m0 = v0 ? m[lane] : zerov<T>(), m1 = v1 ? m[lane + 64] : zerov<T>();
      const double bb = wave_sum(abs2(J0) + abs2(J1));
      T q0, q1;
      if (!group_matvec(m, q0, q1)) { ok = false; break; }
      T r0v = J0 - q0, r1v = J1 - q1, p0 = r0v, p1 = r1v;
      double rr = wave_sum(abs2(r0v) + abs2(r1v));
      const double stop = 1e-28 * bb;
      bool conv = rr <= stop;
      int cgi = 0;
      for (; cgi < 64 && !conv; ++cgi) {
        if (tid < 64) {
          if (v0) pv[lane] = p0;
          if (v1) pv[lane + 64] = p1;
        }
        __syncthreads();
        if (!group_matvec(pv, q0, q1)) { ok = false; break; }
        const double pq = wave_sum(rev(cmul(p0, q0)) + rev(cmul(p1, q1)));
        if (!(pq > 0.0)) break;
        const double alpha = rr / pq;
        m0 += alpha * p0;
        m1 += alpha * p1;
        r0v -= alpha * q0;
        r1v -= alpha * q1;
        const double rn = wave_sum(abs2(r0v) + abs2(r1v));
        const double beta = rn / rr;
        rr = rn;
        conv = rn <= stop;
        p0 = r0v + beta * p0;
        p1 = r1v + beta * p1;
      }
      if (!ok) break;
      cg_iters_total += cgi;
      cg_solves += 1;
      if (!conv) { ok = false; break; }
      // eps = m^H g_s m - 2 Re(m^H J) + N = N - Re(m^H (J + r)), r the residual
      const double eps_est = N - wave_sum(rev(cmul(m0, J0 + r0v)) + rev(cmul(m1, J1 + r1v)));
      if (tid < 64) {
        if (v0) m[lane] = m0;
        if (v1) m[lane + 64] = m1;
      }
      __syncthreads();
      // the new free factor, the fixed one isometric
      for (int e = tid; e < R * Dn; e += blockDim.x) {
        if (half == 0) {
          const int a = e / Dn, j = e % Dn;
          MXs[a * FIT_RMAX + j] = m[a * Dn + j];
          MYs[a * FIT_RMAX + j] = Qf[a * FIT_RMAX + j];
        } else {
          const int j = e / R, b = e % R;
          MYs[b * FIT_RMAX + j] = m[j * R + b];
          MXs[b * FIT_RMAX + j] = Qf[b * FIT_RMAX + j];
        }
      }
      __syncthreads();
      if (lead) tick(2);
      // the residual form loses about log10(N / eps) digits: above 1e-8 N it
      // is kept, below that the error is evaluated directly
      if (eps_est > 1e-8 * N) {
        eps = eps_est;
      } else if (!group_error(eps)) {
        ok = false;
        break;
      }
      if (lead) tick(3);
      if (st && tid == 0) {
        st[16 + 2 * iter + half] = eps;
        st[16 + 2 * fp.n_iter + 2 * iter + half] = tau;
      }
    }
    if (!ok) break;
    iters = iter + 1;
    const bool stop = fp.early_stop && (prev - eps <= fp.conv_tol * N);
    prev = eps;
    if (stop) break;
  }
  if (!ok) {
    redo();
    return;
  }
  if (!lead) return;
  // balancing (the leader), its buffers in the space of the g_s rows
  FitShared<T> Sb;
  Sb.y = y; Sb.MX = MXs; Sb.MY = MYs; Sb.Qf = Qf;
  Sb.sa = gsl; Sb.sv = gsl + FIT_RMAX * FIT_RMAX; Sb.J = gsl + 2 * FIT_RMAX * FIT_RMAX; Sb.m = gsl + 3 * FIT_RMAX * FIT_RMAX;
  Sb.s = sv_s; Sb.red = red; Sb.vec = vec; Sb.idx = nullptr;
  // MX, MY were kept with stride FIT_RMAX over 16 rows: fit_qr_small reads R rows
  __syncthreads();
  const int Dk = fit_balance<T>(D, R, Dn, kappa, Sb, MXo + (size_t)it * R * D, MYo + (size_t)it * R * D, &flag);
  tick(4);
  if (st && tid == 0) {
    st[9] = 3.0;  // certified by the metric repair
    st[15] = cg_solves > 0 ? (double)cg_iters_total / cg_solves : 0.0;
    st[10] = (double)tph0; st[11] = (double)tph1; st[12] = (double)tph2;
    st[13] = (double)tph3; st[14] = (double)tph4;
    st[2] = eps;
    st[3] = N > 0 ? eps / N : 0.0;
    st[5] = Dk;
    st[6] = iters;
    st[7] = 0;
    st[8] = isfinite(eps) && isfinite(N) ? 0.0 : 1.0;
    for (int j = 0; j < D; ++j) st[16 + 4 * fp.n_iter + j] = j < Dk ? Sb.s[j] / Sb.s[0] : 0.0;
  }
}

// control words of every item to zero before a group launch (a kernel, not
// a memset, so that a captured step holds no memset node)
__global__ void k_grp_reset(int batch, unsigned* ctl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch * 4) ctl[(size_t)(i / 4) * GRP_CTL + i % 4] = 0u;
}

hipError_t launch_bond_fit(bool cplx, int batch, int D, int R, const void* g, const void* RX, const void* RY,
                           const FitParams& fp, void* MX, void* MY, double* stats, int stats_stride, void* ws,
                           hipStream_t st, const ProfHook& ph, const double* cert, const void* guess) {
  if (batch <= 0) return hipSuccess;
  if (R > FIT_RMAX || D > FIT_RMAX || R * D > 256) return hipErrorInvalidValue;
  size_t el = cplx ? 16 : 8;
  constexpr size_t LDS_MAX = 160 * 1024 - 16 * 1024;
  // the n x CHOL_BS panel of the certification only for metrics it certifies
  static_assert(FIT_CERT_NMAX == 256 && FAST_NX == 200 && CG_NX == 200, "fit_work_elems");
  size_t shm = fit_shared_fixed_bytes(el, R) + fit_work_elems(R, D) * el + fit_packed_bytes(cplx, R, D);
  ph(PK_FIT, 0);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  // the LDS limit once per device and element type (every call on devices
  // beyond the table)
  static bool attr_set[64][2] = {};
  static int ncu_of[64] = {};
  const bool in_table = dev >= 0 && dev < 64;
  if (!in_table || !attr_set[dev][cplx ? 1 : 0]) {
    // allow the full 160 KiB of LDS for the dynamic part
    e = cplx ? hipFuncSetAttribute((const void*)k_bond_fit<cd>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_MAX)
             : hipFuncSetAttribute((const void*)k_bond_fit<double>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_MAX);
    if (e != hipSuccess) return e;
    e = cplx ? hipFuncSetAttribute((const void*)k_bond_fit_grp<cd>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_MAX)
             : hipFuncSetAttribute((const void*)k_bond_fit_grp<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   LDS_MAX);
    if (e != hipSuccess) return e;
    if (in_table) attr_set[dev][cplx ? 1 : 0] = true;
  }
  if (dev >= 0 && dev < 64 && ncu_of[dev] == 0) {
    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    ncu_of[dev] = ncu;
  }
  if (shm > LDS_MAX) return hipErrorInvalidValue;
  // The group fit for certified items of a Trotter step (metric repair's
  // certificate and the SVDU guess at hand), when every item's members fit
  // on the chip at once (one workgroup per CU): G members per item, at most
  // R, as few as give the same largest share of slabs.
  int G = 0;
  const int b8 = (batch + 7) / 8 * 8;
  if (g && cert && guess && R <= 16 && D <= 8 && R * D <= GRP_NXMAX && D >= GRP_MIN_D && dev >= 0 && dev < 64) {
    const int gmax = std::min(std::min(R, GRP_MAX), ncu_of[dev] / b8);
    if (gmax >= 2) {
      const int nsl = (R + gmax - 1) / gmax;
      G = (R + nsl - 1) / nsl;
      if (grp_shared_bytes(el, R, D, G) > LDS_MAX) G = 0;
    }
  }
  const unsigned* redo = nullptr;
  if (G >= 2) {
    char* base = (char*)ws + align256((size_t)batch * fit_ws_elems(D, R) * el);
    unsigned* ctl = (unsigned*)base;
    base += align256((size_t)batch * GRP_CTL * 4);
    char* xv = base;
    base += align256((size_t)batch * 2 * R * R * el);
    double* xs = (double*)base;
    hipLaunchKernelGGL(k_grp_reset, dim3((batch * 4 + 255) / 256), dim3(256), 0, st, batch, ctl);
    const size_t shg = grp_shared_bytes(el, R, D, G);
    if (cplx)
      hipLaunchKernelGGL(k_bond_fit_grp<cd>, dim3(b8 * G), dim3(FIT_THREADS), shg, st, batch, G, D, R, (const cd*)g,
                         (const cd*)RX, (const cd*)RY, fp, (cd*)MX, (cd*)MY, stats, stats_stride, (cd*)ws, ctl,
                         (cd*)xv, xs, cert, (const cd*)guess);
    else
      hipLaunchKernelGGL(k_bond_fit_grp<double>, dim3(b8 * G), dim3(FIT_THREADS), shg, st, batch, G, D, R,
                         (const double*)g, (const double*)RX, (const double*)RY, fp, (double*)MX, (double*)MY, stats,
                         stats_stride, (double*)ws, ctl, (double*)xv, xs, cert, (const double*)guess);
    redo = ctl;
  }
  if (cplx)
    hipLaunchKernelGGL(k_bond_fit<cd>, dim3(batch), dim3(FIT_THREADS), shm, st, D, R, (const cd*)g, (const cd*)RX,
                       (const cd*)RY, fp, (cd*)MX, (cd*)MY, stats, stats_stride, (cd*)ws, cert, (const cd*)guess, redo);
  else
    hipLaunchKernelGGL(k_bond_fit<double>, dim3(batch), dim3(FIT_THREADS), shm, st, D, R, (const double*)g,
                       (const double*)RX, (const double*)RY, fp, (double*)MX, (double*)MY, stats, stats_stride,
                       (double*)ws, cert, (const double*)guess, redo);
  ph(PK_FIT, 1);
  return hipGetLastError();
}

hipError_t launch_svdu_guess(bool cplx, int batch, int D, int R, const void* RX, const void* RY, double kappa,
                             void* guess, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (R > FIT_RMAX || D > FIT_RMAX) return hipErrorInvalidValue;
  if (cplx)
    hipLaunchKernelGGL(k_svdu_guess<cd>, dim3(batch), dim3(FIT_THREADS), 0, st, D, R, (const cd*)RX, (const cd*)RY,
                       kappa, (cd*)guess);
  else
    hipLaunchKernelGGL(k_svdu_guess<double>, dim3(batch), dim3(FIT_THREADS), 0, st, D, R, (const double*)RX,
                       (const double*)RY, kappa, (double*)guess);
  return hipGetLastError();
}

}  // namespace ntu
