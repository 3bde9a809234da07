// Small dense linear algebra executed by one workgroup (or one thread).
// Used by the gate split, the SVDU guess, the balancing SVD, the metric
// repair and the bond fit.  All FP64.
#pragma once
#include "common.h"

namespace ntu {

// One-sided (Hestenes) Jacobi rotation of the column pair (p, q) that makes
// them orthogonal.  Returns false when they already are (to rounding).
// Given alpha = |c_p|^2, beta = |c_q|^2, gamma = c_p^H c_q, the rotation is
// J = diag(1, e^{-i phi}) [[c, s], [-s, c]] with gamma = |gamma| e^{i phi}.
template <class T>
NTU_DEV bool jacobi_params(double alpha, double beta, T gamma, double& c, double& s, T& e, double gfloor = 0.0) {
  double g = absv(gamma);
  if (!(g > 1e-15 * sqrt(alpha * beta)) || !(g > gfloor)) return false;
  double zeta = (beta - alpha) / (2.0 * g);
  double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  c = 1.0 / sqrt(1.0 + t * t);
  s = c * t;
  e = conjv(phasev(gamma));  // e^{-i phi}
  return true;
}

// Serial one-sided Jacobi SVD of a column-major m x n matrix A (lda >= m):
// on return the columns of A are U_j * s_j (descending s), V (n x n,
// column-major, ldv) holds the right singular vectors: A_in = U S V^H.
template <class T>
NTU_DEV void svd_serial(T* A, int m, int n, int lda, T* V, int ldv, double* s) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) V[i + j * ldv] = realv<T>(i == j ? 1.0 : 0.0);
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rot = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double a = 0, b = 0;
        T g = zerov<T>();
        for (int i = 0; i < m; ++i) {
          a += abs2(A[i + p * lda]);
          b += abs2(A[i + q * lda]);
          g += cmul(A[i + p * lda], A[i + q * lda]);
        }
        double c, sn;
        T e;
        if (!jacobi_params(a, b, g, c, sn, e)) continue;
        rot = true;
        for (int i = 0; i < m; ++i) {
          T x = A[i + p * lda], y = A[i + q * lda] * e;
          A[i + p * lda] = c * x - sn * y;
          A[i + q * lda] = sn * x + c * y;
        }
        for (int i = 0; i < n; ++i) {
          T x = V[i + p * ldv], y = V[i + q * ldv] * e;
          V[i + p * ldv] = c * x - sn * y;
          V[i + q * ldv] = sn * x + c * y;
        }
      }
    if (!rot) break;
  }
  for (int j = 0; j < n; ++j) {
    double a = 0;
    for (int i = 0; i < m; ++i) a += abs2(A[i + j * lda]);
    s[j] = sqrt(a);
  }
  // selection sort, descending
  for (int j = 0; j < n; ++j) {
    int k = j;
    for (int l = j + 1; l < n; ++l)
      if (s[l] > s[k]) k = l;
    if (k != j) {
      double t = s[j]; s[j] = s[k]; s[k] = t;
      for (int i = 0; i < m; ++i) { T x = A[i + j * lda]; A[i + j * lda] = A[i + k * lda]; A[i + k * lda] = x; }
      for (int i = 0; i < n; ++i) { T x = V[i + j * ldv]; V[i + j * ldv] = V[i + k * ldv]; V[i + k * ldv] = x; }
    }
  }
}

// Pairing of round r (0 <= r < n2-1) of the round-robin ("circle") schedule
// over n2 (even) columns: pair k of the round is (first, second), each pair
// disjoint, every unordered pair met once per n2-1 rounds.
NTU_DEV void rr_pair(int n2, int r, int k, int& a, int& b) {
  // player 0 fixed, others rotate (0 <= r < n2 - 1 and 0 <= slot < n2, so
  // one conditional subtraction takes the place of the modulo)
  auto pos = [&](int slot) -> int {
    if (slot == 0) return 0;
    const int x = slot - 1 + r;
    return 1 + (x >= n2 - 1 ? x - (n2 - 1) : x);
  };
  int x = pos(k), y = pos(n2 - 1 - k);
  a = x < y ? x : y;
  b = x < y ? y : x;
}

// Block-parallel one-sided Jacobi SVD of a small column-major m x n matrix in
// shared memory (m <= 32, n <= 32, lda >= m).  One wave per column pair:
// lanes 0..31 carry rows of A, lanes 32..63 rows of V.  On return the columns
// of A are U_j s_j in descending order of s, V the right singular vectors.
// sh_flag: one int of shared memory.  Must be called by the whole block.
template <class T>
NTU_DEV void svd_block_small(T* A, int m, int n, int lda, T* V, int ldv, double* s, int* sh_flag) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  for (int e = tid; e < n * n; e += blockDim.x) {
    int i = e % n, j = e / n;
    V[i + j * ldv] = realv<T>(i == j ? 1.0 : 0.0);
  }
  // Column pairs whose inner product is below (1e-15 ||A||_F)^2 are left
  // alone: such columns are rounding noise of the rotations (their singular
  // values lie below 1e-15 of the largest), and rotating them against each
  // other only makes new noise of the same size, so the sweeps would not end.
  __shared__ double fro2_sh;
  if (tid == 0) {
    double f2 = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < m; ++i) f2 += abs2(A[i + j * lda]);
    fro2_sh = f2;
  }
  __syncthreads();
  const double gfloor = 1e-30 * fro2_sh;
  const int n2 = (n + 1) & ~1;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) *sh_flag = 0;
    __syncthreads();
    for (int r = 0; r < n2 - 1; ++r) {
      for (int k = w; k < n2 / 2; k += nw) {
        int p, q;
        rr_pair(n2, r, k, p, q);
        if (q >= n) continue;  // dummy column of an odd n
        double a = 0, b = 0;
        T g = zerov<T>();
        if (lane < m) {
          T x = A[lane + p * lda], y = A[lane + q * lda];
          a = abs2(x); b = abs2(y); g = cmul(x, y);
        }
        // rows live in lanes 0..31 (m <= 32)
        a = lanes32_sum(a); b = lanes32_sum(b); g = lanes32_sum(g);
        double c, sn;
        T e;
        if (!jacobi_params(a, b, g, c, sn, e, gfloor)) continue;
        if (lane < m) {
          T x = A[lane + p * lda], y = A[lane + q * lda] * e;
          A[lane + p * lda] = c * x - sn * y;
          A[lane + q * lda] = sn * x + c * y;
        } else if (lane >= 32 && lane - 32 < n) {
          int i = lane - 32;
          T x = V[i + p * ldv], y = V[i + q * ldv] * e;
          V[i + p * ldv] = c * x - sn * y;
          V[i + q * ldv] = sn * x + c * y;
        }
        if (lane == 0) *sh_flag = 1;
      }
      __syncthreads();
    }
    int f = *sh_flag;
    __syncthreads();
    if (!f) break;
  }
  if (tid < n) {
    double a = 0;
    for (int i = 0; i < m; ++i) a += abs2(A[i + tid * lda]);
    s[tid] = sqrt(a);
  }
  __syncthreads();
  if (tid == 0) {
    for (int j = 0; j < n; ++j) {
      int k = j;
      for (int l = j + 1; l < n; ++l)
        if (s[l] > s[k]) k = l;
      if (k != j) {
        double t = s[j]; s[j] = s[k]; s[k] = t;
        for (int i = 0; i < m; ++i) { T x = A[i + j * lda]; A[i + j * lda] = A[i + k * lda]; A[i + k * lda] = x; }
        for (int i = 0; i < n; ++i) { T x = V[i + j * ldv]; V[i + j * ldv] = V[i + k * ldv]; V[i + k * ldv] = x; }
      }
    }
  }
  __syncthreads();
}

// In-place Cholesky A = L L^H of an n x n Hermitian matrix (row-major, lda),
// lower triangle overwritten by L (upper triangle left as is).  Returns true
// when every pivot is positive and finite.  Whole block; red: >= 64 doubles.
template <class T>
NTU_DEV bool block_cholesky(T* A, int n, int lda, double* red) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    double piv = rev(A[k * lda + k]);
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (threadIdx.x == 0) bad = 1;
      __syncthreads();
      break;
    }
    double lkk = sqrt(piv), inv = 1.0 / lkk;
    // column k below the diagonal
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[i * lda + k] = A[i * lda + k] * inv;
    __syncthreads();
    if (threadIdx.x == 0) A[k * lda + k] = realv<T>(lkk);
    // trailing update of the lower triangle: A[i][j] -= L[i][k] conj(L[j][k]), k < j <= i
    const int m = n - k - 1;
    const long long tot = (long long)m * (m + 1) / 2;
    for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
      // map e -> (ii, jj) with 0 <= jj <= ii < m (row-wise packing)
      int ii = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while ((long long)(ii + 1) * (ii + 2) / 2 <= e) ++ii;
      while ((long long)ii * (ii + 1) / 2 > e) --ii;
      int jj = (int)(e - (long long)ii * (ii + 1) / 2);
      int i = k + 1 + ii, j = k + 1 + jj;
      A[i * lda + j] = A[i * lda + j] - mulc(A[i * lda + k], A[j * lda + k]);
    }
    __syncthreads();
  }
  bool ok = (bad == 0);
  __syncthreads();
  return ok;
}

// Parallel cyclic two-sided Jacobi eigensolver of an n x n Hermitian matrix
// (row-major, lda; destroyed: on return its diagonal holds the eigenvalues)
// with eigenvectors accumulated in V (row-major, ldv; column j = vector j).
// Round-robin ordering: n/2 disjoint rotations per round.  Whole block.
// pc, ps, pe, pq: shared scratch of >= (n+1)/2 entries each (n <= 2^15).
// JB: entries per thread whose loads are in flight together in the update
// passes (registers: 4 JB values of T for A, 2 JB for V).
template <class T, int JB = (is_cplx<T>::value ? 4 : 8)>
NTU_DEV int block_jacobi_eigh(T* A, int n, int lda, T* V, int ldv, double* pc, double* ps, T* pe,
                              int* pq, int* sh_cnt, double fro) {
  const int tid = threadIdx.x;
  for (long long e = tid; e < (long long)n * n; e += blockDim.x) {
    int i = (int)(e / n), j = (int)(e % n);
    V[i * ldv + j] = realv<T>(i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (n < 2) return 0;
  const int n2 = (n + 1) & ~1, np = n2 / 2;
  const int bq = (int)blockDim.x / np, br = (int)blockDim.x % np;
  // Off-diagonal entries below 1e-14 ||A||_F are left alone.  That is the
  // rounding level of the input itself (a metric summed over thousands of
  // terms in FP64); rotating entries at that level (the mutual entries of a
  // block of zero modes) only makes new ones of the same size, so the sweeps
  // would not end.  Leaving them changes V max(Lambda, 0) V^H by at most their
  // Frobenius norm (the projection onto the non-negative matrices does not
  // increase Frobenius distances).
  const double tiny = 1e-14 * fro;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) *sh_cnt = 0;
    __syncthreads();
    for (int r = 0; r < n2 - 1; ++r) {
      // rotation parameters of every pair of the round from the current A
      for (int k = tid; k < np; k += blockDim.x) {
        int p, q;
        rr_pair(n2, r, k, p, q);
        pq[k] = p | (q << 16);  // the round's pairs for the update passes
        pc[k] = 1.0; ps[k] = 0.0; pe[k] = realv<T>(1.0);
        if (q >= n) continue;
        T apq = A[p * lda + q];
        double g = absv(apq);
        double app = rev(A[p * lda + p]), aqq = rev(A[q * lda + q]);
        if (!(g > 1e-15 * sqrt(fabs(app * aqq))) || !(g > tiny)) continue;
        double zeta = (aqq - app) / (2.0 * g);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t);
        pc[k] = c; ps[k] = c * t; pe[k] = conjv(phasev(apq));  // e^{-i phi}
        atomicAdd(sh_cnt, 1);
      }
      __syncthreads();
      // A <- J^H A J and V <- V J in one pass.  Every entry lies in the 2 x 2
      // block of one pair of pairs (k1 for its row, k2 for its column): the
      // row rotation of k1, row_p' = c row_p - s e^{i phi} row_q, row_q' =
      // s row_p + c e^{i phi} row_q, then the column rotation of k2, col_p' =
      // c col_p - s e^{-i phi} col_q, col_q' = s col_p + c e^{-i phi} col_q
      // (the same operations, in the same order, as a pass over all rows
      // followed by a pass over all columns).  k2 runs fastest over the
      // threads, so a wave touches two rows of A.  Indices >= n belong to the
      // dummy of an odd n and are left out.
      // A thread loads a chunk of JB entries before it updates any of them:
      // taken one at a time, the loads of an entry would wait for the stores
      // of the one before (the compiler cannot rule out that they alias), one
      // memory round trip per entry.  Every entry of a round belongs to one
      // thread, so the order does not change any result.  The pair indices
      // of entry e = k1 np + k2 advance by blockDim.x = bq np + br per step
      // (no integer divisions, which AMDGPU does in software).
      const int na = np * np;
      int k1 = tid / np, k2 = tid % np;
      for (int e0 = tid; e0 < na; e0 += JB * (int)blockDim.x) {
        int K1[JB], K2[JB];
        T ea[JB], eb[JB], ec_[JB], ed[JB];
#pragma unroll
        for (int u = 0; u < JB; ++u) {
          K1[u] = k1; K2[u] = k2;
          k2 += br; k1 += bq;
          if (k2 >= np) { k2 -= np; ++k1; }
        }
#pragma unroll
        for (int u = 0; u < JB; ++u) {
          ea[u] = eb[u] = ec_[u] = ed[u] = zerov<T>();
          if (K1[u] >= np) continue;
          if (ps[K1[u]] == 0.0 && ps[K2[u]] == 0.0) continue;
          const int pq1 = pq[K1[u]], pq2 = pq[K2[u]];
          const int p1 = pq1 & 0xffff, q1 = pq1 >> 16, p2 = pq2 & 0xffff, q2 = pq2 >> 16;
          const bool hq1 = q1 < n, hq2 = q2 < n;
          ea[u] = A[p1 * lda + p2];
          if (hq2) eb[u] = A[p1 * lda + q2];
          if (hq1) ec_[u] = A[q1 * lda + p2];
          if (hq1 && hq2) ed[u] = A[q1 * lda + q2];
        }
#pragma unroll
        for (int u = 0; u < JB; ++u) {
          if (K1[u] >= np) continue;
          const double s1 = ps[K1[u]], s2 = ps[K2[u]];
          if (s1 == 0.0 && s2 == 0.0) continue;
          const int pq1 = pq[K1[u]], pq2 = pq[K2[u]];
          const int p1 = pq1 & 0xffff, q1 = pq1 >> 16, p2 = pq2 & 0xffff, q2 = pq2 >> 16;
          const bool hq1 = q1 < n, hq2 = q2 < n;
          T a = ea[u], b = eb[u], c_ = ec_[u], d_ = ed[u];
          if (s1 != 0.0) {
            const double c = pc[K1[u]];
            const T ec = conjv(pe[K1[u]]);
            T x = a, y = ec * c_;
            a = c * x - s1 * y;
            c_ = s1 * x + c * y;
            x = b; y = ec * d_;
            b = c * x - s1 * y;
            d_ = s1 * x + c * y;
          }
          if (s2 != 0.0) {
            const double c = pc[K2[u]];
            const T ev = pe[K2[u]];
            T x = a, y = b * ev;
            a = c * x - s2 * y;
            b = s2 * x + c * y;
            x = c_; y = d_ * ev;
            c_ = c * x - s2 * y;
            d_ = s2 * x + c * y;
          }
          A[p1 * lda + p2] = a;
          if (hq2) A[p1 * lda + q2] = b;
          if (hq1) A[q1 * lda + p2] = c_;
          if (hq1 && hq2) A[q1 * lda + q2] = d_;
        }
      }
      // V <- V J: entry e = i np + k, row i, pair k; the same stepping
      const int nv = n * np;
      int vi = tid / np, vk = tid % np;
      for (int e0 = tid; e0 < nv; e0 += JB * (int)blockDim.x) {
        int I[JB], K[JB];
        T vx[JB], vy[JB];
#pragma unroll
        for (int u = 0; u < JB; ++u) {
          I[u] = vi; K[u] = vk;
          vk += br; vi += bq;
          if (vk >= np) { vk -= np; ++vi; }
        }
#pragma unroll
        for (int u = 0; u < JB; ++u) {
          vx[u] = vy[u] = zerov<T>();
          if (I[u] >= n || ps[K[u]] == 0.0) continue;
          const int pqk = pq[K[u]];
          vx[u] = V[I[u] * ldv + (pqk & 0xffff)];
          vy[u] = V[I[u] * ldv + (pqk >> 16)];
        }
#pragma unroll
        for (int u = 0; u < JB; ++u) {
          if (I[u] >= n || ps[K[u]] == 0.0) continue;
          const int pqk = pq[K[u]];
          const double c = pc[K[u]], s = ps[K[u]];
          const T x = vx[u], y = vy[u] * pe[K[u]];
          V[I[u] * ldv + (pqk & 0xffff)] = c * x - s * y;
          V[I[u] * ldv + (pqk >> 16)] = s * x + c * y;
        }
      }
      __syncthreads();
    }
    int cnt = *sh_cnt;
    __syncthreads();
    if (cnt == 0) return sweep + 1;
  }
  return 40;
}

// Offset of entry (i, j) of a symmetric matrix stored as its lower triangle,
// row by row.
NTU_DEV int packed_at(int i, int j) { return i >= j ? ((i * (i + 1)) >> 1) + j : ((j * (j + 1)) >> 1) + i; }

// block_jacobi_eigh for a real symmetric n x n matrix held packed in shared
// memory (Ap: n (n + 1) / 2 doubles, lower triangle row by row; on return its
// diagonal holds the eigenvalues), eigenvectors into VT transposed (VT[j ldv
// + i] = component i of vector j; global memory).  The same rotations,
// round-robin ordering, skip and
// stopping rules.  The update J^T A J takes each unordered pair of pairs
// (k1 >= k2) once: the block of the other order is the transpose of this one
// and shares its storage, and a diagonal block (k1 = k2) keeps its one
// off-diagonal entry.  The pairs of a round depend only on its number, so
// each round's parameter pass also writes the next round's pairs, and the
// entries of V that a round rotates are loaded at its start: their latency
// runs under the parameter pass and the update of A.  Entry u of a thread is
// (pair, row) = divmod(tid + u blockDim, n), the same in every round (a wave
// reads and writes consecutive components of one vector); the
// first VB are loaded ahead (registers: the kernels that use this stay within
// 256 VGPRs at VB = 8), any further ones after the update of A.  A round
// without any rotation (most rounds of the last sweeps) skips both updates:
// rc (two shared ints) counts the rotations of the current and the next
// round.  pq: 2 (n + 1) / 2 ints.  Whole block.
template <int VB = 8>
NTU_DEV int block_jacobi_eigh_packed(double* Ap, int n, double* VT, int ldv, double* pc, double* ps, int* pq,
                                     int* sh_cnt, int* rc, double fro) {
  const int tid = threadIdx.x;
  for (long long e = tid; e < (long long)n * n; e += blockDim.x) {
    int i = (int)(e / n), j = (int)(e % n);
    VT[i * ldv + j] = i == j ? 1.0 : 0.0;
  }
  if (n < 2) {
    __syncthreads();
    return 0;
  }
  const int n2 = (n + 1) & ~1, np = n2 / 2, ntri = np * (np + 1) / 2;
  const int bq = (int)blockDim.x / np, br = (int)blockDim.x % np;
  const double tiny = 1e-14 * fro;
  int* pq_cur = pq;
  int* pq_nxt = pq + np;
  for (int k = tid; k < np; k += blockDim.x) {
    int p, q;
    rr_pair(n2, 0, k, p, q);
    pq_cur[k] = p | (q << 16);
  }
  if (tid == 0) rc[0] = rc[1] = 0;
  // this thread's first entry of V: pair vk0, row vi0 (the others follow by
  // steps of blockDim: rows advance by ri, pairs by rk)
  const int vk0 = tid / n, vi0 = tid % n;
  const int rk = (int)blockDim.x / n, ri = (int)blockDim.x % n;
  __syncthreads();
  const int rounds = n2 - 1;
  int gr = 0;  // rounds so far over all sweeps: its parity selects the counter
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) *sh_cnt = 0;
    __syncthreads();
    for (int r = 0; r < rounds; ++r) {
      // entries of V this round rotates (their pairs are known already)
      double vx[VB], vy[VB];
      {
        int vi = vi0, vk = vk0;
#pragma unroll
        for (int u = 0; u < VB; ++u) {
          const int pqk = pq_cur[min(vk, np - 1)];
          vx[u] = VT[(pqk & 0xffff) * ldv + vi];
          vy[u] = VT[min(pqk >> 16, n - 1) * ldv + vi];
          vi += ri; vk += rk;
          if (vi >= n) { vi -= n; ++vk; }
        }
      }
      // rotation parameters of this round; the next round's pairs
      const int rn = r + 1 < rounds ? r + 1 : 0;
      for (int k = tid; k < np; k += blockDim.x) {
        int p, q;
        rr_pair(n2, rn, k, p, q);
        pq_nxt[k] = p | (q << 16);
        const int pqk = pq_cur[k];
        p = pqk & 0xffff; q = pqk >> 16;
        pc[k] = 1.0; ps[k] = 0.0;
        if (q >= n) continue;
        const double apq = Ap[packed_at(q, p)];
        const double g = fabs(apq);
        const double app = Ap[packed_at(p, p)], aqq = Ap[packed_at(q, q)];
        if (!(g > 1e-15 * sqrt(fabs(app * aqq))) || !(g > tiny)) continue;
        const double zeta = (aqq - app) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        // the sign of apq (the phase of the complex form) folded into s
        pc[k] = c; ps[k] = (apq < 0.0 ? -c : c) * t;
        atomicAdd(&rc[gr & 1], 1);
      }
      __syncthreads();
      // every thread reads this round's count; the next round's counter is
      // cleared (nobody touches it before the barrier that ends this round)
      const int nrot = rc[gr & 1];
      if (tid == 0) {
        *sh_cnt += nrot;
        rc[(gr + 1) & 1] = 0;
      }
      ++gr;
      if (nrot == 0) {
        int* t = pq_cur; pq_cur = pq_nxt; pq_nxt = t;
        __syncthreads();
        continue;
      }
      // A <- J^T A J on the blocks k1 >= k2, TB at a time: all their pair
      // data, then all their entries, then the rotations (the identity for
      // a pair that does not rotate) and the stores of what changed
      constexpr int TB = 3;
      for (int e0 = tid; e0 < ntri; e0 += TB * (int)blockDim.x) {
        int k1[TB], k2[TB];
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          const int e = min(e0 + u * (int)blockDim.x, ntri - 1);
          int x = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
          x -= ((x * (x + 1)) >> 1) > e ? 1 : 0;
          x += (((x + 1) * (x + 2)) >> 1) <= e ? 1 : 0;
          k1[u] = x;
          k2[u] = e - ((x * (x + 1)) >> 1);
        }
        int pq1[TB], pq2[TB];
        double c1[TB], s1[TB], c2[TB], s2[TB];
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          pq1[u] = pq_cur[k1[u]]; pq2[u] = pq_cur[k2[u]];
          c1[u] = pc[k1[u]]; s1[u] = ps[k1[u]];
          c2[u] = pc[k2[u]]; s2[u] = ps[k2[u]];
        }
        double ea[TB], eb[TB], ec_[TB], ed[TB];
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          const int p1 = pq1[u] & 0xffff, q1 = min(pq1[u] >> 16, n - 1);
          const int p2 = pq2[u] & 0xffff, q2 = min(pq2[u] >> 16, n - 1);
          ea[u] = Ap[packed_at(p1, p2)];
          eb[u] = Ap[packed_at(p1, q2)];
          ec_[u] = Ap[packed_at(q1, p2)];
          ed[u] = Ap[packed_at(q1, q2)];
        }
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          // row rotation of pair k1, then column rotation of pair k2
          double a = c1[u] * ea[u] - s1[u] * ec_[u];
          double c_ = s1[u] * ea[u] + c1[u] * ec_[u];
          double b = c1[u] * eb[u] - s1[u] * ed[u];
          double d_ = s1[u] * eb[u] + c1[u] * ed[u];
          const double a2 = c2[u] * a - s2[u] * b, b2 = s2[u] * a + c2[u] * b;
          const double c2_ = c2[u] * c_ - s2[u] * d_, d2 = s2[u] * c_ + c2[u] * d_;
          const bool live = e0 + u * (int)blockDim.x < ntri && (s1[u] != 0.0 || s2[u] != 0.0);
          if (live) {
            const int p1 = pq1[u] & 0xffff, q1 = pq1[u] >> 16, p2 = pq2[u] & 0xffff, q2 = pq2[u] >> 16;
            const bool hq1 = q1 < n, hq2 = q2 < n;
            Ap[packed_at(p1, p2)] = a2;
            if (hq2) Ap[packed_at(p1, q2)] = b2;
            // on a diagonal block (q1, p2) is (p2, q1) = (p1, q2), stored above
            if (hq1 && k1[u] != k2[u]) Ap[packed_at(q1, p2)] = c2_;
            if (hq1 && hq2) Ap[packed_at(q1, q2)] = d2;
          }
        }
      }
      // V <- V J: the entries loaded at the start of the round, then the
      // rest in batches of VB (loaded here)
      {
        int vi = vi0, vk = vk0;
        for (int b = 0; vk < np; ++b) {
          if (b > 0) {
            int wi = vi, wk = vk;
#pragma unroll
            for (int u = 0; u < VB; ++u) {
              const int pqk = pq_cur[min(wk, np - 1)];
              vx[u] = VT[(pqk & 0xffff) * ldv + wi];
              vy[u] = VT[min(pqk >> 16, n - 1) * ldv + wi];
              wi += ri; wk += rk;
              if (wi >= n) { wi -= n; ++wk; }
            }
          }
#pragma unroll
          for (int u = 0; u < VB; ++u) {
            const double s = vk < np ? ps[vk] : 0.0;
            if (s != 0.0) {
              const int pqk = pq_cur[vk];
              const double c = pc[vk];
              VT[(pqk & 0xffff) * ldv + vi] = c * vx[u] - s * vy[u];
              VT[(pqk >> 16) * ldv + vi] = s * vx[u] + c * vy[u];
            }
            vi += ri; vk += rk;
            if (vi >= n) { vi -= n; ++vk; }
          }
        }
      }
      int* t = pq_cur; pq_cur = pq_nxt; pq_nxt = t;
      __syncthreads();
    }
    int cnt = *sh_cnt;
    __syncthreads();
    if (cnt == 0) return sweep + 1;
  }
  return 40;
}

}  // namespace ntu



namespace ntu {

NTU_DEV void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Blocked right-looking Cholesky A = L L^H of an n x n Hermitian matrix held
// row-major in global memory (lower triangle read and overwritten by L).
// Per block column of width BS: the panel (rows k0..n-1) is staged in shared
// memory, wave 0 factors the diagonal block, every thread solves panel rows,
// and the trailing lower triangle gets a rank-BS update in 4 x 4 register
// tiles.  pan: shared T[n * BS]; flag: one shared int.  Returns false
// (uniformly) on a non-positive or non-finite pivot.  Whole block.
// ---------------------------------------------------------------------------
template <class T, int BS>
NTU_DEV bool blocked_cholesky(T* A, int n, int lda, T* pan, int* flag) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += BS) {
    const int bs = min(BS, n - k0), m = n - k0;
    for (int e = tid; e < m * bs; e += nt) {
      const int i = e / bs, c = e % bs;
      pan[i * BS + c] = (i < c) ? zerov<T>() : A[(size_t)(k0 + i) * lda + k0 + c];
    }
    __syncthreads();
    if (wv == 0) {
      for (int c = 0; c < bs; ++c) {
        const double piv = rev(pan[c * BS + c]);
        if (!(piv > 0.0) || !isfinite(piv)) {
          if (lane == 0) *flag = 1;
          break;
        }
        const double lcc = sqrt(piv), inv = 1.0 / lcc;
        if (lane > c && lane < bs) pan[lane * BS + c] = pan[lane * BS + c] * inv;
        wave_sync_lds();
        if (lane == c) pan[c * BS + c] = realv<T>(lcc);
        const int w2 = bs - 1 - c;
        for (int e = lane; e < w2 * w2; e += 64) {
          const int r = c + 1 + e / w2, q = c + 1 + e % w2;
          if (q <= r) pan[r * BS + q] -= mulc(pan[r * BS + c], pan[q * BS + c]);
        }
        wave_sync_lds();
      }
    }
    __syncthreads();
    if (*flag) return false;
    // panel rows below the diagonal block: L_i. = A_i. L_kk^{-H}
    for (int i = bs + tid; i < m; i += nt) {
      for (int c = 0; c < bs; ++c) {
        T v = pan[i * BS + c];
        for (int q = 0; q < c; ++q) v -= mulc(pan[i * BS + q], pan[c * BS + q]);
        pan[i * BS + c] = v * (1.0 / rev(pan[c * BS + c]));
      }
    }
    __syncthreads();
    for (int e = tid; e < m * bs; e += nt) {
      const int i = e / bs, c = e % bs;
      if (i >= c) A[(size_t)(k0 + i) * lda + k0 + c] = pan[i * BS + c];
    }
    // trailing update, lower triangle of rows/cols k0 + bs .. n-1, in 4 x 4 tiles
    const int mt = m - bs, tt = (mt + 3) / 4;
    const int ntile = tt * (tt + 1) / 2;
    for (int t = tid; t < ntile; t += nt) {
      int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
      while (ti * (ti + 1) / 2 > t) --ti;
      const int tj = t - ti * (ti + 1) / 2;
      T acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = zerov<T>();
      for (int c = 0; c < bs; ++c) {
        T li[4], lj[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int i = bs + 4 * ti + a, j = bs + 4 * tj + a;
          li[a] = i < m ? pan[i * BS + c] : zerov<T>();
          lj[a] = j < m ? pan[j * BS + c] : zerov<T>();
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += mulc(li[a], lj[b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = 4 * ti + a, j = 4 * tj + b;
          if (i < mt && j <= i) {
            T* p = &A[(size_t)(k0 + bs + i) * lda + k0 + bs + j];
            *p = *p - acc[a][b];
          }
        }
    }
    __syncthreads();
  }
  return true;
}

// Solve L L^H x = b with the factor of blocked_cholesky (L in the lower
// triangle of A, global).  b, x: shared, length n (b is overwritten).
// Whole block.
template <class T, int BS>
NTU_DEV void blocked_chol_solve(const T* A, int n, int lda, T* b, T* x, T* dblk) {
  const int tid = threadIdx.x, nt = blockDim.x;
  // forward: L z = b, z stored in b
  for (int k0 = 0; k0 < n; k0 += BS) {
    const int bs = min(BS, n - k0);
    for (int e = tid; e < bs * bs; e += nt) dblk[e] = A[(size_t)(k0 + e / bs) * lda + k0 + e % bs];
    __syncthreads();
    if (tid == 0) {
      for (int c = 0; c < bs; ++c) {
        const int r = k0 + c;
        T v = b[r];
        for (int q = 0; q < c; ++q) v -= dblk[c * bs + q] * b[k0 + q];
        b[r] = v * (1.0 / rev(dblk[c * bs + c]));
      }
    }
    __syncthreads();
    for (int i = k0 + bs + tid; i < n; i += nt) {
      T v = b[i];
      for (int c = 0; c < bs; ++c) v -= A[(size_t)i * lda + k0 + c] * b[k0 + c];
      b[i] = v;
    }
    __syncthreads();
  }
  // backward: L^H x = z
  const int nb = (n + BS - 1) / BS;
  for (int kb = nb - 1; kb >= 0; --kb) {
    const int k0 = kb * BS, bs = min(BS, n - k0);
    for (int e = tid; e < bs * bs; e += nt) dblk[e] = A[(size_t)(k0 + e / bs) * lda + k0 + e % bs];
    __syncthreads();
    if (tid == 0) {
      for (int c = bs - 1; c >= 0; --c) {
        const int r = k0 + c;
        T v = b[r];
        for (int q = c + 1; q < bs; ++q) v -= cmul(dblk[q * bs + c], x[k0 + q]);
        x[r] = v * (1.0 / rev(dblk[c * bs + c]));
      }
    }
    __syncthreads();
    for (int i = tid; i < k0; i += nt) {
      T v = b[i];
      for (int c = 0; c < bs; ++c) v -= cmul(A[(size_t)(k0 + c) * lda + i], x[k0 + c]);
      b[i] = v;
    }
    __syncthreads();
  }
}

// Gershgorin certification of g: every eigenvalue lies in the union of the
// discs |lambda - g_ii| <= sum_{j != i} |g_ij|, so lo = min_i (g_ii - r_i)
// bounds lambda_min from below and hi = max_i (g_ii + r_i) bounds lambda_max
// from above.  Certified if lo > margin * hi.  Whole block; red: >=
// max(n, blockDim.x) doubles of shared memory.
template <class T>
NTU_DEV bool gershgorin_certify(const T* __restrict__ G, int n, double margin, double* red) {
  // Hermitian G: the off-diagonal absolute row sum of row r equals that of
  // column r, read with r fastest (coalesced).  Work item (r, part) sums a
  // range of rows c; parts meet in red.
  const int tid = threadIdx.x, parts = max(1, (int)blockDim.x / n), cs = (n + parts - 1) / parts;
  double lo = INFINITY, hi = -INFINITY;
  for (int wi = tid; wi < parts * n; wi += blockDim.x) {
    const int r = wi % n, part = wi / n;
    const int c1 = min(n, (part + 1) * cs);
    double off = 0.0;
    for (int c0 = part * cs; c0 < c1; c0 += 8) {
      T v[8];
#pragma unroll
      for (int l = 0; l < 8; ++l) v[l] = c0 + l < c1 ? G[(size_t)(c0 + l) * n + r] : zerov<T>();
#pragma unroll
      for (int l = 0; l < 8; ++l)
        if (c0 + l < c1 && c0 + l != r) off += sqrt(abs2(v[l]));
    }
    red[wi] = off;
  }
  __syncthreads();
  for (int r = tid; r < n; r += blockDim.x) {
    double off = 0.0;
    for (int part = 0; part < parts; ++part) off += red[part * n + r];
    const double dg = rev(G[(size_t)r * n + r]);
    lo = fmin(lo, dg - off);
    hi = fmax(hi, dg + off);
  }
  lo = -block_max(-lo, red);
  hi = block_max(hi, red);
  return lo > 0.0 && hi > 0.0 && lo > margin * hi;
}

}  // namespace ntu
