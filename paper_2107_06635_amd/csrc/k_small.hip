// Gate split (Fig. 2(a)), reduction + QR (Fig. 2(b)), recombination
// (Fig. 2(e)) and the 90-degree rotation of site tensors.
#include "kernels.h"
#include "fastdiv.h"
#include "linalg.h"
#include <algorithm>

namespace ntu {

// ---------------------------------------------------------------------------
// Gate split: operator SVD of the regrouped gate, one workgroup per item.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(64) k_gate_split(int d, int rg, const T* gate, T* GA, T* GB,
                                                   double* sigma) {
  constexpr int NMAX = 16;
  __shared__ T A[NMAX * NMAX];
  __shared__ T V[NMAX * NMAX];
  __shared__ double s[NMAX];
  const int n = d * d, it = blockIdx.x;
  const T* G = gate + (size_t)it * n * n;
  // M[(s1' s1), (s2' s2)] = G[(s1' s2'), (s1 s2)], stored column-major
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    int row = e / n, col = e % n;
    int s1p = row / d, s1 = row % d, s2p = col / d, s2 = col % d;
    A[row + col * n] = G[(s1p * d + s2p) * n + s1 * d + s2];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    svd_serial<T>(A, n, n, n, V, n, s);
    for (int k = 0; k < n; ++k) {
      // U column = A column / s; phase: first entry within 1e-8 of the max modulus real positive
      double inv = s[k] > 0 ? 1.0 / s[k] : 0.0;
      double mx = 0;
      for (int i = 0; i < n; ++i) mx = fmax(mx, absv(A[i + k * n]));
      T ph = realv<T>(1.0);
      for (int i = 0; i < n; ++i) {
        double m = absv(A[i + k * n]);
        if (m >= (1.0 - 1e-8) * mx && m > 0) {
          ph = conjv(phasev(A[i + k * n]));
          break;
        }
      }
      for (int i = 0; i < n; ++i) {
        A[i + k * n] = A[i + k * n] * ph * inv;
        V[i + k * n] = V[i + k * n] * ph;
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * rg; e += blockDim.x) {
    int row = e / rg, k = e % rg;  // row = (s' s)
    double sq = sqrt(s[k]);
    GA[(size_t)it * n * rg + e] = A[row + k * n] * sq;
    GB[(size_t)it * n * rg + e] = conjv(V[row + k * n]) * sq;
  }
  for (int e = threadIdx.x; e < n; e += blockDim.x) sigma[(size_t)it * n + e] = s[e];
}

hipError_t launch_gate_split(bool cplx, int batch, int d, int rg, const void* gate, void* GA, void* GB,
                             double* sigma, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (cplx)
    hipLaunchKernelGGL(k_gate_split<cd>, dim3(batch), dim3(64), 0, st, d, rg, (const cd*)gate, (cd*)GA,
                       (cd*)GB, sigma);
  else
    hipLaunchKernelGGL(k_gate_split<double>, dim3(batch), dim3(64), 0, st, d, rg, (const double*)gate,
                       (double*)GA, (double*)GB, sigma);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Action rho -> G rho G^dagger of a spin-1/2 two-site gate on the products of
// the Hermitian basis O = (X, Y, Z, 1) (Eq. 11, Fig. 8):
//   S[(a' b'), (a b)] = Tr((O^a' x O^b') G (O^a x O^b) G^dagger) / 4.
// Each basis product is a signed permutation matrix: row (i1 i2) holds one
// entry, phase ph_a(i1) ph_b(i2) in {+-1, +-i}, at column (pi_a(i1),
// pi_b(i2)).  With P' = O^a' x O^b' and P = O^a x O^b the trace is
//   sum_{i,k} ph'(i) G[pi'(i), k] ph(k) conj(G[i, pi(k)]),
// sixteen products of two gate entries.  One thread per output entry, one
// workgroup of 256 per item.
// ---------------------------------------------------------------------------
NTU_DEV int pauli_col(int a, int i) { return (a <= 1) ? 1 - i : i; }
// phase of the entry of row i of basis operator a, as (re, im)
NTU_DEV cd pauli_phase(int a, int i) {
  switch (a) {
    case 1: return i == 0 ? cd{0.0, -1.0} : cd{0.0, 1.0};  // Y
    case 2: return i == 0 ? cd{1.0, 0.0} : cd{-1.0, 0.0};  // Z
    default: return cd{1.0, 0.0};                          // X, 1
  }
}
NTU_DEV cd gate_entry(const double* G, int r, int c) { return cd{G[r * 4 + c], 0.0}; }
NTU_DEV cd gate_entry(const cd* G, int r, int c) { return G[r * 4 + c]; }

template <class T>
__global__ void __launch_bounds__(256) k_superop(const T* __restrict__ gate, double* __restrict__ S) {
  const int it = blockIdx.x, e = threadIdx.x;
  const int row = e >> 4, col = e & 15;
  const int ap = row >> 2, bp = row & 3, a = col >> 2, b = col & 3;
  const T* G = gate + (size_t)it * 16;
  cd acc{0.0, 0.0};
  for (int i = 0; i < 4; ++i) {
    const int i1 = i >> 1, i2 = i & 1;
    const int pi_p = pauli_col(ap, i1) * 2 + pauli_col(bp, i2);
    const cd php = pauli_phase(ap, i1) * pauli_phase(bp, i2);
    for (int k = 0; k < 4; ++k) {
      const int k1 = k >> 1, k2 = k & 1;
      const int pi_k = pauli_col(a, k1) * 2 + pauli_col(b, k2);
      const cd ph = pauli_phase(a, k1) * pauli_phase(b, k2);
      acc += php * gate_entry(G, pi_p, k) * ph * conjv(gate_entry(G, i, pi_k));
    }
  }
  S[(size_t)it * 256 + e] = 0.25 * acc.x;
}

hipError_t launch_superop(bool cplx_gate, int batch, const void* gate, double* S, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (cplx_gate)
    hipLaunchKernelGGL(k_superop<cd>, dim3(batch), dim3(256), 0, st, (const cd*)gate, S);
  else
    hipLaunchKernelGGL(k_superop<double>, dim3(batch), dim3(256), 0, st, (const double*)gate, S);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reduction: W = gate factor applied to the site tensor, then Gram-Schmidt QR
// with the projection applied twice and the rank rule.  One workgroup per item.
// ---------------------------------------------------------------------------
template <class T> NTU_DEV T load_site(const double* p, long long i) { return realv<T>(p[i]); }
// a site value as loaded, in the compute type
template <class T> NTU_DEV T widen_site(double v) { return realv<T>(v); }
template <class T> NTU_DEV T widen_site(cd v) { return v; }
template <class T> NTU_DEV T widen_site(float2 v) { return cd{(double)v.x, (double)v.y}; }
template <class T> NTU_DEV T load_site(const cd* p, long long i);
template <> NTU_DEV cd load_site<cd>(const cd* p, long long i) { return p[i]; }
template <class T> NTU_DEV T load_site(const float2* p, long long i);
template <> NTU_DEV cd load_site<cd>(const float2* p, long long i) {
  float2 v = p[i];
  return cd{(double)v.x, (double)v.y};
}

// W = (gate factor) x (site tensor), row-major nrow x R, for the Gram-Schmidt
// reductions: row (s', a, t, i3, i4) with s' the gate's output index, column
// (q, k) with q the bond index and k the gate's rank index; X side: (l, b) =
// (i3, i4), bond r = q; Y side: (b, r) = (i3, i4), bond l = q.  A thread takes
// whole rows and decodes a row's indices once in 32-bit arithmetic (AMDGPU
// divides in software, 64-bit divisions far more slowly); each entry sums over
// s in the same order as a per-entry loop would.
template <class T, class S>
NTU_DEV void form_w(const S* __restrict__ X, const T* __restrict__ G, int d, int na, int D, int rg, int side,
                    int nrow, T* __restrict__ Qi) {
  const int R = D * rg, D2 = D * D, D3 = D2 * D;
  const long long D4 = (long long)D3 * D;
  for (int row = threadIdx.x; row < nrow; row += blockDim.x) {
    const int i4 = row % D, i3 = (row / D) % D, t = (row / D2) % D;
    const int pa = row / D3, sp = pa / na, a = pa % na;
    for (int q = 0; q < D; ++q) {
      const long long inner = side == 0 ? (long long)(i3 * D2 + i4 * D + q) : (long long)(q * D2 + i3 * D + i4);
      for (int k = 0; k < rg; ++k) {
        T v = zerov<T>();
        for (int s = 0; s < d; ++s)
          v += G[(sp * d + s) * rg + k] * load_site<T>(X, (long long)(s * na + a) * D4 + (long long)t * D3 + inner);
        Qi[(size_t)row * R + q * rg + k] = v;
      }
    }
  }
}

constexpr int QR_THREADS = 256;
constexpr int QR_RMAX = 32;

// The Y side of a launch that reduces both sides of a bond at once
// (grid.y = 2); unused with grid.y = 1.
template <class T, class S> struct ReduceY {
  const S* site;
  const T* gf;
  T* Q;
  T* R;
};

template <class T, class S>
__global__ void __launch_bounds__(QR_THREADS) k_reduce_qr(int d, int na, int D, int rg, const S* site,
                                                         const T* gf, long long gf_stride, int side, T* Q, T* Rm,
                                                         double kappa, const int* todo, ReduceY<T, S> yside) {
  __shared__ double red[16 * 64];
  __shared__ double hv[2 * QR_RMAX];
  __shared__ double cacc[2 * QR_RMAX];
  constexpr int NC = is_cplx<T>::value ? 2 : 1;
  if (blockIdx.y == 1) {  // the Y side of a two-sided launch
    site = yside.site; gf = yside.gf; Q = yside.Q; Rm = yside.R; side = 1;
  }
  const int it = blockIdx.x, tid = threadIdx.x, ti = blockIdx.y * gridDim.x + blockIdx.x;
  if (todo && todo[ti] == 0) return;  // done by the Cholesky QR
  const int p = d * na, R = D * rg;
  const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D3 * D;
  const long long nrow = p * D3;
  const S* X = site + (size_t)it * p * D4;
  const T* G = gf + (size_t)it * gf_stride;
  T* Qi = Q + (size_t)it * nrow * R;
  T* Ri = Rm + (size_t)it * R * R;

  // 1. W into Q (row-major nrow x R)
  form_w<T, S>(X, G, d, na, D, rg, side, (int)nrow, Qi);
  for (int e = tid; e < R * R; e += blockDim.x) Ri[e] = zerov<T>();
  __syncthreads();

  // 2. largest column norm
  double part[QR_RMAX];
#pragma unroll
  for (int j = 0; j < QR_RMAX; ++j) part[j] = 0.0;
  for (long long row = tid; row < nrow; row += blockDim.x)
#pragma unroll
    for (int j = 0; j < QR_RMAX; ++j)
      if (j < R) part[j] += abs2(Qi[row * R + j]);
  block_sum_vec(part, R, red, hv);
  double scale = 0.0;
  for (int j = 0; j < R; ++j) scale = fmax(scale, sqrt(hv[j]));
  __syncthreads();

  // 3. Gram-Schmidt, projection twice
  for (int j = 0; j < R; ++j) {
    for (int i = tid; i < 2 * QR_RMAX; i += blockDim.x) cacc[i] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      double hp[2 * QR_RMAX];
#pragma unroll
      for (int i = 0; i < 2 * QR_RMAX; ++i) hp[i] = 0.0;
      for (long long row = tid; row < nrow; row += blockDim.x) {
        T qj = Qi[row * R + j];
#pragma unroll
        for (int i = 0; i < QR_RMAX; ++i)
          if (i < j) {
            T h = cmul(Qi[row * R + i], qj);
            hp[NC * i] += rev(h);
            if (NC == 2) hp[NC * i + 1] += imv(h);
          }
      }
      block_sum_vec(hp, NC * j, red, hv);
      for (long long row = tid; row < nrow; row += blockDim.x) {
        T v = Qi[row * R + j];
        for (int i = 0; i < j; ++i) {
          T h;
          if constexpr (NC == 2) h = T{hv[2 * i], hv[2 * i + 1]};
          else h = realv<T>(hv[i]);
          v -= Qi[row * R + i] * h;
        }
        Qi[row * R + j] = v;
      }
      if (tid < NC * j) cacc[tid] += hv[tid];
      __syncthreads();
    }
    double nn = 0.0;
    for (long long row = tid; row < nrow; row += blockDim.x) nn += abs2(Qi[row * R + j]);
    nn = sqrt(block_sum(nn, red));
    const bool keep = scale > 0.0 && nn > kappa * scale;
    const double inv = keep ? 1.0 / nn : 0.0;
    for (long long row = tid; row < nrow; row += blockDim.x) Qi[row * R + j] = Qi[row * R + j] * inv;
    if (tid == 0) {
      Ri[j * R + j] = realv<T>(keep ? nn : 0.0);
      for (int i = 0; i < j; ++i) {
        if constexpr (NC == 2) Ri[i * R + j] = T{cacc[2 * i], cacc[2 * i + 1]};
        else Ri[i * R + j] = realv<T>(cacc[i]);
      }
    }
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// The same Gram-Schmidt QR with W held in registers: thread t of NT owns
// rows t, t + NT, ... (RPT of them, R <= QRR_RMAX columns each), so each
// projection pass is register arithmetic plus one block reduction of a fixed
// number of partial sums, with no sweep over W in memory.  Taken for real
// types when the rows fit (p D^3 <= RPT NT with the configurations of
// reduce_launch); same steps, projection twice, same rank rule.
// ---------------------------------------------------------------------------
constexpr int QRR_RMAX = 16;

// n partial sums per thread (registers) summed over the block into out[0..n)
template <int N> NTU_DEV void block_sum_fixed(const double (&vals)[N], double* red, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double v = wave_sum(vals[i]);
    if (lane == 0) red[w * 64 + i] = v;
    __builtin_amdgcn_sched_barrier(0);  // one reduction at a time (register pressure)
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double sum = 0.0;
    for (int k = 0; k < nw; ++k) sum += red[k * 64 + i];
    out[i] = sum;
  }
  __syncthreads();
}

template <class T, class S, int RPT, int NT>
__global__ void __launch_bounds__(NT) k_reduce_qr_reg(int d, int na, int D, int rg, const S* site,
                                                              const T* gf, long long gf_stride, int side, T* Q,
                                                              T* Rm, double kappa, const int* todo,
                                                              ReduceY<T, S> yside) {
  constexpr int NC = is_cplx<T>::value ? 2 : 1, RM = QRR_RMAX;
  __shared__ double red[16 * 64];
  __shared__ double hv[NC * RM];
  __shared__ double cacc[NC * RM];
  if (blockIdx.y == 1) {  // the Y side of a two-sided launch
    site = yside.site; gf = yside.gf; Q = yside.Q; Rm = yside.R; side = 1;
  }
  const int it = blockIdx.x, tid = threadIdx.x, ti = blockIdx.y * gridDim.x + blockIdx.x;
  if (todo && todo[ti] == 0) return;  // done by the Cholesky QR
  const int p = d * na, R = D * rg;
  const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D3 * D;
  const long long nrow = p * D3;
  const S* X = site + (size_t)it * p * D4;
  const T* G = gf + (size_t)it * gf_stride;
  T* Qi = Q + (size_t)it * nrow * R;
  T* Ri = Rm + (size_t)it * R * R;
  for (int e = tid; e < R * R; e += blockDim.x) Ri[e] = zerov<T>();

  // 1. W into Q (row-major nrow x R), then this thread's rows into registers
  form_w<T, S>(X, G, d, na, D, rg, side, (int)nrow, Qi);
  __syncthreads();
  T w[RPT][RM];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const long long row = tid + (long long)k * NT;
#pragma unroll
    for (int j = 0; j < RM; ++j) w[k][j] = (row < nrow && j < R) ? Qi[row * R + j] : zerov<T>();
  }

  // 2. largest column norm
  double part[RM];
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    part[j] = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) part[j] += abs2(w[k][j]);
  }
  block_sum_fixed<RM>(part, red, hv);
  double scale = 0.0;
  for (int j = 0; j < R; ++j) scale = fmax(scale, sqrt(hv[j]));

  // 3. Gram-Schmidt, projection twice (column j picked out of the registers
  // by comparison, so that every index into w stays a constant)
  for (int j = 0; j < R; ++j) {
    if (tid < NC * RM) cacc[tid] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      double hp[NC * RM];
#pragma unroll
      for (int i = 0; i < NC * RM; ++i) hp[i] = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        T qj = zerov<T>();
#pragma unroll
        for (int i = 0; i < RM; ++i)
          if (i == j) qj = w[k][i];
#pragma unroll
        for (int i = 0; i < RM; ++i)
          if (i < j) {
            const T h = cmul(w[k][i], qj);
            hp[NC * i] += rev(h);
            if constexpr (NC == 2) hp[NC * i + 1] += imv(h);
          }
      }
      block_sum_fixed<NC * RM>(hp, red, hv);
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        T v = zerov<T>();
#pragma unroll
        for (int i = 0; i < RM; ++i)
          if (i == j) v = w[k][i];
#pragma unroll
        for (int i = 0; i < RM; ++i)
          if (i < j) {
            T h;
            if constexpr (NC == 2) h = T{hv[2 * i], hv[2 * i + 1]};
            else h = realv<T>(hv[i]);
            v -= w[k][i] * h;
            // keeps the next coefficient's load below this use, so that the
            // coefficients are not all held in registers beside the rows
            __builtin_amdgcn_sched_barrier(0);
          }
#pragma unroll
        for (int i = 0; i < RM; ++i)
          if (i == j) w[k][i] = v;
      }
      if (tid < NC * j) cacc[tid] += hv[tid];
    }
    double nn[1] = {0.0};
#pragma unroll
    for (int k = 0; k < RPT; ++k)
#pragma unroll
      for (int i = 0; i < RM; ++i)
        if (i == j) nn[0] += abs2(w[k][i]);
    block_sum_fixed<1>(nn, red, hv);
    const double norm = sqrt(hv[0]);
    const bool keep = scale > 0.0 && norm > kappa * scale;
    const double inv = keep ? 1.0 / norm : 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k)
#pragma unroll
      for (int i = 0; i < RM; ++i)
        if (i == j) w[k][i] = w[k][i] * inv;
    if (tid == 0) {
      Ri[j * R + j] = realv<T>(keep ? norm : 0.0);
      for (int i = 0; i < j; ++i) {
        if constexpr (NC == 2) Ri[i * R + j] = T{cacc[2 * i], cacc[2 * i + 1]};
        else Ri[i * R + j] = realv<T>(cacc[i]);
      }
    }
  }

  // 4. Q rows
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const long long row = tid + (long long)k * NT;
    if (row < nrow)
#pragma unroll
      for (int j = 0; j < RM; ++j)
        if (j < R) Qi[row * R + j] = w[k][j];
  }
}

// ---------------------------------------------------------------------------
// Reduction by Cholesky QR, applied twice (three sweeps over W instead of two
// per column).  W is formed in chunks of rows staged in shared memory; the
// Gram matrix W^H W = R1^H R1 gives Q1 = W R1^{-1}, and the same step on Q1
// gives Q = Q1 R2^{-1}, R = R2 R1.  Taken only when every pivot of the first
// factorisation exceeds (CQR_PIV * max_j |W_j|)^2: then every column is far
// above the rank threshold, the Gram matrix resolves the factor to rounding,
// and the result is the same QR (real positive diagonal) as Gram-Schmidt.
// Otherwise todo[it] = 1 and the Gram-Schmidt kernel takes the item.
// ---------------------------------------------------------------------------
constexpr int CQR_THREADS = 512;
constexpr int CQR_RMAX = 24;        // largest R on this path
constexpr int CQR_CH = 128;         // rows per chunk
constexpr int CQR_LD = CQR_RMAX + 1;
constexpr double CQR_PIV = 1e-6;

// Upper Cholesky factor Rf of the Hermitian n x n matrix G (G = Rf^H Rf) and
// its inverse Ti, all row-major with stride CQR_RMAX.  Wave 0 (threadIdx.x <
// 64); returns whether every pivot exceeds floor2 (same value on all lanes).
template <class T, int LDM = CQR_RMAX>
NTU_DEV bool cqr_chol(const T* G, int n, double floor2, T* Rf, T* Ti) {
  const int lane = threadIdx.x;
  for (int e = lane; e < LDM * LDM; e += 64) {
    Rf[e] = zerov<T>();
    Ti[e] = zerov<T>();
  }
  wave_sync_lds();
  bool good = true;
  for (int k = 0; k < n; ++k) {
    T sv = zerov<T>();
    if (lane >= k && lane < n) {
      sv = G[k * LDM + lane];
      for (int i = 0; i < k; ++i) sv -= cmul(Rf[i * LDM + k], Rf[i * LDM + lane]);
    }
    const double piv = __shfl(rev(sv), k, 64);
    good = good && piv > floor2 && isfinite(piv);
    const double rkk = good ? sqrt(piv) : 1.0;
    if (lane == k) Rf[k * LDM + k] = realv<T>(rkk);
    else if (lane > k && lane < n) Rf[k * LDM + lane] = sv * (1.0 / rkk);
    wave_sync_lds();
  }
  if (lane < n) {
    const int j = lane;
    Ti[j * LDM + j] = realv<T>(1.0 / rev(Rf[j * LDM + j]));
    for (int i = j - 1; i >= 0; --i) {
      T acc = zerov<T>();
      for (int l = i + 1; l <= j; ++l) acc += Rf[i * LDM + l] * Ti[l * LDM + j];
      Ti[i * LDM + j] = acc * (-1.0 / rev(Rf[i * LDM + i]));
    }
  }
  wave_sync_lds();
  return good;
}

template <class T, class S>
__global__ void __launch_bounds__(CQR_THREADS) k_reduce_cholqr(int d, int na, int D, int rg, const S* site,
                                                              const T* gf, long long gf_stride, int side, T* Q,
                                                              T* Rm, double kappa, int* todo, ReduceY<T, S> yside) {
  __shared__ T ch[CQR_CH * CQR_LD];
  __shared__ T ch2[CQR_CH * CQR_LD];
  __shared__ T G[CQR_RMAX * CQR_RMAX];
  __shared__ T R1[CQR_RMAX * CQR_RMAX];
  __shared__ T T1[CQR_RMAX * CQR_RMAX];
  __shared__ T R2[CQR_RMAX * CQR_RMAX];
  __shared__ T T2[CQR_RMAX * CQR_RMAX];
  __shared__ int ok;
  if (blockIdx.y == 1) {  // the Y side of a two-sided launch
    site = yside.site; gf = yside.gf; Q = yside.Q; Rm = yside.R; side = 1;
  }
  const int it = blockIdx.x, tid = threadIdx.x, nt = blockDim.x, ti = blockIdx.y * gridDim.x + blockIdx.x;
  const int p = d * na, R = D * rg;
  if (R > CQR_RMAX) {
    if (tid == 0) todo[ti] = 1;
    return;
  }
  const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D3 * D;
  const int nrow = (int)(p * D3);
  const S* X = site + (size_t)it * p * D4;
  const T* Gf = gf + (size_t)it * gf_stride;
  T* Qi = Q + (size_t)it * nrow * R;
  T* Ri = Rm + (size_t)it * R * R;
  constexpr int NG = (CQR_RMAX * CQR_RMAX + CQR_THREADS - 1) / CQR_THREADS;  // Gram entries per thread
  T acc[NG];

  // sweep over the rows of `src` (global, row-major nrow x R) or of W:
  // stage each chunk, optionally multiply by the upper triangular Tm, write
  // the result back to Qi, and accumulate its Gram matrix into G.
  auto sweep = [&](int mode, const T* Tm) {
#pragma unroll
    for (int u = 0; u < NG; ++u) acc[u] = zerov<T>();
    for (int c0 = 0; c0 < nrow; c0 += CQR_CH) {
      const int rows = min(CQR_CH, nrow - c0);
      for (int e = tid; e < rows * R; e += nt) {
        const int rl = e / R, col = e % R;
        const int row = c0 + rl;
        T v;
        if (mode == 0) {
          const int q = col / rg, k = col % rg;
          const int i4 = row % D, i3 = (row / D) % D, t = (row / (int)D2) % D;
          const int pa = row / (int)D3, sp = pa / na, a = pa % na;
          v = zerov<T>();
          for (int s = 0; s < d; ++s) {
            const long long base = (long long)(s * na + a) * D4 + t * D3;
            const long long off = side == 0 ? base + i3 * D2 + i4 * D + q : base + q * D2 + i3 * D + i4;
            v += Gf[(sp * d + s) * rg + k] * load_site<T>(X, off);
          }
        } else {
          v = Qi[(size_t)row * R + col];
        }
        ch[rl * CQR_LD + col] = v;
      }
      __syncthreads();
      T* src = ch;
      if (mode != 0) {
        for (int e = tid; e < rows * R; e += nt) {
          const int rl = e / R, j = e % R;
          T v = zerov<T>();
          for (int i = 0; i <= j; ++i) v += ch[rl * CQR_LD + i] * Tm[i * CQR_RMAX + j];
          ch2[rl * CQR_LD + j] = v;
        }
        __syncthreads();
        src = ch2;
      }
      for (int e = tid; e < rows * R; e += nt) Qi[(size_t)(c0 + e / R) * R + e % R] = src[(e / R) * CQR_LD + e % R];
#pragma unroll
      for (int u = 0; u < NG; ++u) {
        const int e = tid + u * nt;
        if (mode != 2 && e < R * R) {
          const int i = e / R, j = e % R;
          T a = acc[u];
          for (int r = 0; r < rows; ++r) a += cmul(src[r * CQR_LD + i], src[r * CQR_LD + j]);
          acc[u] = a;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < NG; ++u) {
      const int e = tid + u * nt;
      if (e < R * R) G[(e / R) * CQR_RMAX + e % R] = acc[u];
    }
    __syncthreads();
  };

  // 1. W and its Gram matrix; first factor
  sweep(0, nullptr);
  if (tid < 64) {
    double mx = 0;
    for (int j = 0; j < R; ++j) mx = fmax(mx, rev(G[j * CQR_RMAX + j]));
    const double piv = fmax(CQR_PIV, 1e3 * kappa);
    const bool g1 = mx > 0 && cqr_chol<T>(G, R, piv * piv * mx, R1, T1);
    if (tid == 0) ok = g1 ? 1 : 0;
  }
  __syncthreads();
  if (!ok) {
    if (tid == 0) todo[ti] = 1;
    return;
  }
  __syncthreads();
  // 2. Q1 = W R1^{-1} and its Gram matrix; second factor (pivots near 1)
  sweep(1, T1);
  if (tid < 64) {
    const bool g2 = cqr_chol<T>(G, R, 0.25, R2, T2);
    if (tid == 0) ok = g2 ? 1 : 0;
  }
  __syncthreads();
  if (!ok) {
    if (tid == 0) todo[ti] = 1;
    return;
  }
  // 3. Q = Q1 R2^{-1} (Gram not needed), R = R2 R1
  sweep(2, T2);
  for (int e = tid; e < R * R; e += nt) {
    const int i = e / R, j = e % R;
    T v = zerov<T>();
    for (int l = i; l <= j; ++l) v += R2[i * CQR_RMAX + l] * R1[l * CQR_RMAX + j];
    Ri[e] = v;
  }
  if (tid == 0) todo[ti] = 0;
}

// ---------------------------------------------------------------------------
// The same Cholesky QR, applied twice, on the FP64 matrix cores for R <= 16,
// with W never stored: forming an entry again from the site tensor costs d
// products, less than storing the p D^3 x R matrix and reading it back, so
// each of the three sweeps forms W again, chunk by chunk in shared memory:
//   sweep 1: G1 = W^H W              -> R1 (pivot test), T1 = R1^{-1}
//   sweep 2: Q1 = W T1, G2 = Q1^H Q1 -> R2, T2 = R2^{-1}
//   sweep 3: Q = W (T1 T2), written once;  R = R2 R1.
// Gram matrices: each wave adds 16 x 16 x 4 products over its K chunks of
// rows (complex: four real products, A = conj(W)^T and B = W taken from the
// same register), and the eight waves' sums are added in shared memory in a
// fixed order.  Right products: one 16-row tile per wave, complex as four
// real products.  Same pivot rule as k_reduce_cholqr.
// ---------------------------------------------------------------------------
constexpr int RQM_CH = 128;  // rows per chunk: eight waves x 16
constexpr int RQM_LD = 17;   // elements per staged row (16 + 1 against bank conflicts)

// divisors of the row and column decoding, fixed at launch
struct RqDiv {
  FastDiv D, D2, D3, na, rg;
};

template <class T, class S>
__global__ void __launch_bounds__(512) k_reduce_cqr_mfma(int d, int na, int D, int rg, const S* site, const T* gf,
                                                        long long gf_stride, int side, T* Q, T* Rm, double kappa,
                                                        int* todo, ReduceY<T, S> yside, RqDiv dv,
                                                        int stage_site) {
  constexpr bool CPLX = is_cplx<T>::value;
  constexpr int CQR_RMAX = 16;  // leading dimension of the small matrices here
  __shared__ T gfs[32];
  __shared__ T Wc[RQM_CH * RQM_LD];  // the chunk: W, then its product (each wave its own 16 rows)
  __shared__ T Gm[CQR_RMAX * CQR_RMAX];
  __shared__ T R1[CQR_RMAX * CQR_RMAX];
  __shared__ T T1[CQR_RMAX * CQR_RMAX];
  __shared__ T R2[CQR_RMAX * CQR_RMAX];
  __shared__ T T2[CQR_RMAX * CQR_RMAX];
  __shared__ T Tt[CQR_RMAX * CQR_RMAX];
  __shared__ int ok;
  // the item's site tensor, when the launch gives it room (stage_site)
  extern __shared__ uint4 site_lds[];  // 16-byte aligned
  if (blockIdx.y == 1) {  // the Y side of a two-sided launch
    site = yside.site; gf = yside.gf; Q = yside.Q; Rm = yside.R; side = 1;
  }
  const int it = blockIdx.x, tid = threadIdx.x, ti = blockIdx.y * gridDim.x + blockIdx.x;
  const int lane = tid & 63, w = tid >> 6, l16 = lane & 15, lk = lane >> 4;
  const int p = d * na, R = D * rg;
  const int D2 = D * D, D3 = D2 * D;
  const long long D4 = (long long)D3 * D;
  const int nrow = p * D3;
  const S* X = site + (size_t)it * p * D4;
  const T* Gf = gf + (size_t)it * gf_stride;
  T* Qi = Q + (size_t)it * nrow * R;
  T* Ri = Rm + (size_t)it * R * R;

  // the gate factor (d d r_g <= 32 entries) in shared memory
  if (tid < d * d * rg) gfs[tid] = Gf[tid];
  // the whole site tensor in shared memory (one pass of 16-byte loads, all
  // in flight), so that the three sweeps form W without global loads
  const S* Xsrc = X;
  if (stage_site) {
    const long long nb = (long long)p * D4 * sizeof(S) / 16;
    const uint4* src = (const uint4*)X;
    uint4* dst = site_lds;
    for (long long e = tid; e < nb; e += blockDim.x) dst[e] = src[e];
    Xsrc = (const S*)site_lds;
  }
  // W rows [c0, c0 + rows) into Wc (zero beyond rows and R): thread t takes
  // row t / 4 and the columns t % 4 + 4 u; d <= 2 site values per entry,
  // loaded raw (load_chunk) a chunk ahead of their use (store_chunk)
  const int rl = tid >> 2, cq = tid & 3;
  S raw[4][2];
  auto load_chunk = [&](int c0) {
    const unsigned row = (unsigned)min(c0 + rl, nrow - 1);
    const unsigned i4 = fmod_(row, dv.D), i3 = fmod_(fdiv(row, dv.D), dv.D), tt = fmod_(fdiv(row, dv.D2), dv.D);
    const unsigned pa = fdiv(row, dv.D3), a = fmod_(pa, dv.na);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const unsigned col = (unsigned)min(cq + 4 * u, R - 1), q = fdiv(col, dv.rg);
      const long long inner = side == 0 ? (long long)(i3 * D2 + i4 * D + q) : (long long)(q * D2 + i3 * D + i4);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int sc = min(s, d - 1);
        raw[u][s] = Xsrc[(long long)(sc * na + a) * D4 + (long long)tt * D3 + inner];
      }
    }
  };
  auto store_chunk = [&](int c0, int rows) {
    const unsigned row = (unsigned)min(c0 + rl, nrow - 1);
    const unsigned sp = fdiv(fdiv(row, dv.D3), dv.na);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int col = cq + 4 * u;
      const unsigned k = fmod_((unsigned)min(col, R - 1), dv.rg);
      T acc = zerov<T>();
#pragma unroll
      for (int s = 0; s < 2; ++s)
        if (s < d) acc += gfs[(sp * d + s) * rg + k] * widen_site<T>(raw[u][s]);
      Wc[rl * RQM_LD + col] = (rl < rows && col < R) ? acc : zerov<T>();
    }
  };
  // the wave's share of a Gram matrix of the staged chunk src
  f64x4 gre, gim;
  auto gram_chunk = [&](const T* src) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const T v = src[(4 * (w + 8 * m) + lk) * RQM_LD + l16];
      if constexpr (CPLX) {
        gre = __builtin_amdgcn_mfma_f64_16x16x4f64(v.x, v.x, gre, 0, 0, 0);
        gre = __builtin_amdgcn_mfma_f64_16x16x4f64(v.y, v.y, gre, 0, 0, 0);
        gim = __builtin_amdgcn_mfma_f64_16x16x4f64(v.x, v.y, gim, 0, 0, 0);
        gim = __builtin_amdgcn_mfma_f64_16x16x4f64(-v.y, v.x, gim, 0, 0, 0);
      } else {
        gre = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, gre, 0, 0, 0);
      }
    }
  };
  // the eight waves' sums into Gm (Pc as scratch); whole block
  auto gram_reduce = [&]() {
    // 8 waves x (re[, im]) x 256 doubles: 32 KiB complex, 16 KiB real, within Pc
    constexpr int NP = CPLX ? 2 : 1;
    double* sc = (double*)Wc;  // free after the sweep's last chunk
    static_assert(8 * NP * 256 * sizeof(double) <= sizeof(T) * RQM_CH * RQM_LD, "scratch of the Gram sums");
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = (lk + 4 * v) * 16 + l16;
      sc[(w * NP + 0) * 256 + e] = gre[v];
      if constexpr (CPLX) sc[(w * NP + 1) * 256 + e] = gim[v];
    }
    __syncthreads();
    if (tid < 256) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < 8; ++k) {
        sr += sc[(k * NP + 0) * 256 + tid];
        if constexpr (CPLX) si += sc[(k * NP + 1) * 256 + tid];
      }
      const int i = tid >> 4, j = tid & 15;
      if (i < R && j < R) {
        if constexpr (CPLX) Gm[i * CQR_RMAX + j] = T{sr, si};
        else Gm[i * CQR_RMAX + j] = sr;
      }
    }
    __syncthreads();
  };
  // this wave's 16-row tile of Wc times the upper triangular Tm (operands
  // from registers tb) -> Pc, or Q at chunk row offset c0
  T tb[4];
  auto load_tb = [&](const T* Tm) {
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int k = 4 * kc + lk;
      tb[kc] = (k < R && l16 < R) ? Tm[k * CQR_RMAX + l16] : zerov<T>();
    }
  };
  auto product_chunk = [&](int c0, int rows, bool to_global) {
    f64x4 pr = {0.0, 0.0, 0.0, 0.0}, pi = {0.0, 0.0, 0.0, 0.0};
    T av[4];  // the wave's rows read before they are overwritten
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) av[kc] = Wc[(16 * w + l16) * RQM_LD + 4 * kc + lk];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const T a = av[kc];
      if constexpr (CPLX) {
        pr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, tb[kc].x, pr, 0, 0, 0);
        pr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, tb[kc].y, pr, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, tb[kc].y, pi, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, tb[kc].x, pi, 0, 0, 0);
      } else {
        pr = __builtin_amdgcn_mfma_f64_16x16x4f64(a, tb[kc], pr, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rl = 16 * w + lk + 4 * v;
      T val;
      if constexpr (CPLX) val = T{pr[v], pi[v]};
      else val = pr[v];
      if (to_global) {
        if (rl < rows && l16 < R) Qi[(size_t)(c0 + rl) * R + l16] = val;
      } else {
        Wc[rl * RQM_LD + l16] = val;  // this wave's own rows
      }
    }
  };
  auto zero_acc = [&]() {
    gre = f64x4{0.0, 0.0, 0.0, 0.0};
    gim = f64x4{0.0, 0.0, 0.0, 0.0};
  };

  // sweep 1: Gram of W, first factor
  __syncthreads();  // gfs
  zero_acc();
  load_chunk(0);
  for (int c0 = 0; c0 < nrow; c0 += RQM_CH) {
    store_chunk(c0, min(RQM_CH, nrow - c0));
    __syncthreads();
    load_chunk(c0 + RQM_CH);
    gram_chunk(Wc);
    __syncthreads();
  }
  gram_reduce();
  if (tid < 64) {
    double mx = 0;
    for (int j = 0; j < R; ++j) mx = fmax(mx, rev(Gm[j * CQR_RMAX + j]));
    const double piv = fmax(CQR_PIV, 1e3 * kappa);
    const bool g1 = mx > 0 && cqr_chol<T, CQR_RMAX>(Gm, R, piv * piv * mx, R1, T1);
    if (tid == 0) ok = g1 ? 1 : 0;
  }
  __syncthreads();
  if (!ok) {
    if (tid == 0) todo[ti] = 1;
    return;
  }
  // sweep 2: Q1 = W T1 and its Gram matrix, second factor (pivots near 1)
  load_tb(T1);
  zero_acc();
  load_chunk(0);
  for (int c0 = 0; c0 < nrow; c0 += RQM_CH) {
    const int rows = min(RQM_CH, nrow - c0);
    store_chunk(c0, rows);
    __syncthreads();
    load_chunk(c0 + RQM_CH);
    product_chunk(c0, rows, false);
    __syncthreads();
    gram_chunk(Wc);
    __syncthreads();
  }
  gram_reduce();
  if (tid < 64) {
    const bool g2 = cqr_chol<T, CQR_RMAX>(Gm, R, 0.25, R2, T2);
    if (tid == 0) ok = g2 ? 1 : 0;
  }
  __syncthreads();
  if (!ok) {
    if (tid == 0) todo[ti] = 1;
    return;
  }
  // T = T1 T2 (upper triangular), R = R2 R1
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e / R, j = e % R;
    T t = zerov<T>(), r = zerov<T>();
    for (int l = i; l <= j; ++l) {
      t += T1[i * CQR_RMAX + l] * T2[l * CQR_RMAX + j];
      r += R2[i * CQR_RMAX + l] * R1[l * CQR_RMAX + j];
    }
    Tt[i * CQR_RMAX + j] = t;
    Ri[e] = r;
  }
  for (int e = tid; e < CQR_RMAX * CQR_RMAX; e += blockDim.x)
    if (e / CQR_RMAX >= R || e % CQR_RMAX >= R || e / CQR_RMAX > e % CQR_RMAX) Tt[e] = zerov<T>();
  __syncthreads();
  // sweep 3: Q = W T
  load_tb(Tt);
  load_chunk(0);
  for (int c0 = 0; c0 < nrow; c0 += RQM_CH) {
    const int rows = min(RQM_CH, nrow - c0);
    store_chunk(c0, rows);
    __syncthreads();
    load_chunk(c0 + RQM_CH);
    product_chunk(c0, rows, true);
    __syncthreads();
  }
  if (tid == 0) todo[ti] = 0;
}

// ---------------------------------------------------------------------------
// The same Cholesky QR, twice, with W formed once and kept in registers for
// the three sweeps.  Wave w holds rows [w 4 KPW, (w + 1) 4 KPW) in the
// operand layout of the 16 x 16 x 4 FP64 Gram products (register c of lane l:
// row 4 c + l / 16 of the wave's block, column l % 16), so both Gram
// matrices are formed straight from registers.  The right products need the
// transposed layout (rows along the lanes of a 16-lane row): a 16-row tile
// passes through a 16 x 16 buffer of the wave's own in shared memory, and
// the product comes back in the Gram layout, ready for the second Gram
// matrix and for coalesced stores of Q.  Needs R <= 16, d <= 2 and p D^3 <=
// 32 KPW rows.
// ---------------------------------------------------------------------------
template <class T, class S, int KPW>
__global__ void __launch_bounds__(512) k_reduce_cqr_reg(int d, int na, int D, int rg, const S* site, const T* gf,
                                                       long long gf_stride, int side, T* Q, T* Rm, double kappa,
                                                       int* todo, ReduceY<T, S> yside, RqDiv dv, int stage_site) {
  constexpr bool CPLX = is_cplx<T>::value;
  constexpr int CQR_RMAX = 16;  // leading dimension of the small matrices here
  __shared__ T gfs[32];
  __shared__ T tbuf[8][16 * 17];  // per wave: one 16 x 16 tile (leading dimension 17)
  __shared__ double gsum[8 * 2 * 256];
  __shared__ T Gm[CQR_RMAX * CQR_RMAX];
  __shared__ T R1[CQR_RMAX * CQR_RMAX];
  __shared__ T T1[CQR_RMAX * CQR_RMAX];
  __shared__ T R2[CQR_RMAX * CQR_RMAX];
  __shared__ T T2[CQR_RMAX * CQR_RMAX];
  __shared__ T Tt[CQR_RMAX * CQR_RMAX];
  __shared__ int ok;
  extern __shared__ uint4 site_lds[];  // the item's site tensor when stage_site (16-byte aligned)
  if (blockIdx.y == 1) {  // the Y side of a two-sided launch
    site = yside.site; gf = yside.gf; Q = yside.Q; Rm = yside.R; side = 1;
  }
  const int it = blockIdx.x, tid = threadIdx.x, ti = blockIdx.y * gridDim.x + blockIdx.x;
  const int lane = tid & 63, w = tid >> 6, l16 = lane & 15, lk = lane >> 4;
  const int p = d * na, R = D * rg;
  const int D2 = D * D, D3 = D2 * D;
  const long long D4 = (long long)D3 * D;
  const int nrow = p * D3;
  const int base = w * 4 * KPW;
  const S* X = site + (size_t)it * p * D4;
  const T* Gf = gf + (size_t)it * gf_stride;
  T* Qi = Q + (size_t)it * nrow * R;
  T* Ri = Rm + (size_t)it * R * R;
  if (tid < d * d * rg) gfs[tid] = Gf[tid];
  const S* Xsrc = X;
  if (stage_site) {
    const long long nb = (long long)p * D4 * sizeof(S) / 16;
    const uint4* src = (const uint4*)X;
    for (long long e = tid; e < nb; e += blockDim.x) site_lds[e] = src[e];
    Xsrc = (const S*)site_lds;
  }
  __syncthreads();
  // W in registers: wr[c] = W[base + 4 c + lk][l16] (zero beyond nrow and R),
  // formed four chunks at a time (their loads in flight together)
  T wr[KPW];
  {
    const unsigned col = (unsigned)min(l16, R - 1), q = fdiv(col, dv.rg), k = fmod_(col, dv.rg);
    const bool colok = l16 < R;
#pragma unroll
    for (int c0 = 0; c0 < KPW; c0 += 4) {
      S raw[4][2];
      unsigned spv[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const unsigned row = (unsigned)min(base + 4 * (c0 + c) + lk, nrow - 1);
        const unsigned i4 = fmod_(row, dv.D), i3 = fmod_(fdiv(row, dv.D), dv.D), tt = fmod_(fdiv(row, dv.D2), dv.D);
        const unsigned pa = fdiv(row, dv.D3), a = fmod_(pa, dv.na);
        spv[c] = fdiv(pa, dv.na);
        const long long inner = side == 0 ? (long long)(i3 * D2 + i4 * D + q) : (long long)(q * D2 + i3 * D + i4);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int sc = min(s, d - 1);
          raw[c][s] = Xsrc[(long long)(sc * na + a) * D4 + (long long)tt * D3 + inner];
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T acc = zerov<T>();
#pragma unroll
        for (int s = 0; s < 2; ++s)
          if (s < d) acc += gfs[(spv[c] * d + s) * rg + k] * widen_site<T>(raw[c][s]);
        const int row = base + 4 * (c0 + c) + lk;
        wr[c0 + c] = (row < nrow && colok) ? acc : zerov<T>();
      }
    }
  }
  f64x4 gre = {0.0, 0.0, 0.0, 0.0}, gim = {0.0, 0.0, 0.0, 0.0};
  auto gram_add = [&](const T& v) {
    if constexpr (CPLX) {
      gre = __builtin_amdgcn_mfma_f64_16x16x4f64(v.x, v.x, gre, 0, 0, 0);
      gre = __builtin_amdgcn_mfma_f64_16x16x4f64(v.y, v.y, gre, 0, 0, 0);
      gim = __builtin_amdgcn_mfma_f64_16x16x4f64(v.x, v.y, gim, 0, 0, 0);
      gim = __builtin_amdgcn_mfma_f64_16x16x4f64(-v.y, v.x, gim, 0, 0, 0);
    } else {
      gre = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, gre, 0, 0, 0);
    }
  };
  // the eight waves' sums into Gm (fixed order); whole block
  auto gram_reduce = [&]() {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = (lk + 4 * v) * 16 + l16;
      gsum[(w * 2 + 0) * 256 + e] = gre[v];
      gsum[(w * 2 + 1) * 256 + e] = CPLX ? gim[v] : 0.0;
    }
    __syncthreads();
    if (tid < 256) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < 8; ++k) {
        sr += gsum[(k * 2 + 0) * 256 + tid];
        si += gsum[(k * 2 + 1) * 256 + tid];
      }
      const int i = tid >> 4, j = tid & 15;
      if (i < R && j < R) {
        if constexpr (CPLX) Gm[i * CQR_RMAX + j] = T{sr, si};
        else Gm[i * CQR_RMAX + j] = sr;
      }
    }
    __syncthreads();
  };
  // tile t of the wave (registers 4 t .. 4 t + 3) times the upper triangular
  // matrix whose B operands are tb: the product in the Gram layout (pv[v]:
  // row 16 t + 4 v + lk, column l16)
  T tb[4];
  auto load_tb = [&](const T* Tm) {
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int kk = 4 * kc + lk;
      tb[kc] = (kk < R && l16 < R) ? Tm[kk * CQR_RMAX + l16] : zerov<T>();
    }
  };
  T* tw = tbuf[w];
  auto tile_product = [&](int t, T (&pv)[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) tw[(4 * v + lk) * 17 + l16] = wr[4 * t + v];
    wave_sync_lds();
    T av[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) av[kc] = tw[l16 * 17 + 4 * kc + lk];
    wave_sync_lds();
    f64x4 pr = {0.0, 0.0, 0.0, 0.0}, pi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      if constexpr (CPLX) {
        pr = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kc].x, tb[kc].x, pr, 0, 0, 0);
        pr = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[kc].y, tb[kc].y, pr, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kc].x, tb[kc].y, pi, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kc].y, tb[kc].x, pi, 0, 0, 0);
      } else {
        pr = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kc], tb[kc], pr, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if constexpr (CPLX) pv[v] = T{pr[v], pi[v]};
      else pv[v] = pr[v];
    }
  };

  // sweep 1: Gram of W, first factor
#pragma unroll
  for (int c = 0; c < KPW; ++c) gram_add(wr[c]);
  gram_reduce();
  if (tid < 64) {
    double mx = 0;
    for (int j = 0; j < R; ++j) mx = fmax(mx, rev(Gm[j * CQR_RMAX + j]));
    const double piv = fmax(CQR_PIV, 1e3 * kappa);
    const bool g1 = mx > 0 && cqr_chol<T, CQR_RMAX>(Gm, R, piv * piv * mx, R1, T1);
    if (tid == 0) ok = g1 ? 1 : 0;
  }
  __syncthreads();
  if (!ok) {
    if (tid == 0) todo[ti] = 1;
    return;
  }
  // sweep 2: Q1 = W T1 tile by tile, its Gram matrix from the products
  load_tb(T1);
  gre = f64x4{0.0, 0.0, 0.0, 0.0};
  gim = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < KPW / 4; ++t) {
    T pv[4];
    tile_product(t, pv);
#pragma unroll
    for (int v = 0; v < 4; ++v) gram_add(pv[v]);
  }
  gram_reduce();
  if (tid < 64) {
    const bool g2 = cqr_chol<T, CQR_RMAX>(Gm, R, 0.25, R2, T2);
    if (tid == 0) ok = g2 ? 1 : 0;
  }
  __syncthreads();
  if (!ok) {
    if (tid == 0) todo[ti] = 1;
    return;
  }
  // T = T1 T2 (upper triangular), R = R2 R1
  for (int e = tid; e < CQR_RMAX * CQR_RMAX; e += blockDim.x) {
    const int i = e / CQR_RMAX, j = e % CQR_RMAX;
    T t = zerov<T>(), r = zerov<T>();
    if (i < R && j < R)
      for (int l = i; l <= j; ++l) {
        t += T1[i * CQR_RMAX + l] * T2[l * CQR_RMAX + j];
        r += R2[i * CQR_RMAX + l] * R1[l * CQR_RMAX + j];
      }
    Tt[e] = t;
    if (i < R && j < R) Ri[i * R + j] = r;
  }
  __syncthreads();
  // sweep 3: Q = W T, stored row by row
  load_tb(Tt);
#pragma unroll
  for (int t = 0; t < KPW / 4; ++t) {
    T pv[4];
    tile_product(t, pv);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = base + 16 * t + 4 * v + lk;
      if (row < nrow && l16 < R) Qi[(size_t)row * R + l16] = pv[v];
    }
  }
  if (tid == 0) todo[ti] = 0;
}

template <class T, class S>
static void reduce_launch(int batch, int sides, int d, int na, int D, int rg, const void* site, const void* gf,
                          long long gf_stride, int side, void* Q, void* R, const void* site_y, const void* gf_y,
                          void* Q_y, void* R_y, double kappa, int* todo, hipStream_t st) {
  const ReduceY<T, S> y{(const S*)site_y, (const T*)gf_y, (T*)Q_y, (T*)R_y};
  const dim3 g(batch, sides);
  if (todo) {
    if (D * rg <= 16 && d <= 2 && d * d * rg <= 32) {
      const RqDiv dv{make_fastdiv(D), make_fastdiv(D * D), make_fastdiv(D * D * D), make_fastdiv(na), make_fastdiv(rg)};
      // the site tensor in shared memory when it takes at most 64 KiB (and
      // its size is a multiple of 16 bytes)
      const size_t site_bytes = (size_t)d * na * D * D * D * D * sizeof(S);
      const int stage = site_bytes <= 64 * 1024 && site_bytes % 16 == 0 ? 1 : 0;
      const long long nrow = (long long)d * na * D * D * D;
      // W in registers when its rows fit the eight waves (32 complex or 64
      // real registers per lane), else staged chunk by chunk
      constexpr int KPW = is_cplx<T>::value ? 32 : 64;
      if (nrow <= 32LL * KPW)
        hipLaunchKernelGGL((k_reduce_cqr_reg<T, S, KPW>), g, dim3(512), stage ? site_bytes : 0, st, d, na, D, rg,
                           (const S*)site, (const T*)gf, gf_stride, side, (T*)Q, (T*)R, kappa, todo, y, dv, stage);
      else
        hipLaunchKernelGGL((k_reduce_cqr_mfma<T, S>), g, dim3(512), stage ? site_bytes : 0, st, d, na, D, rg,
                           (const S*)site, (const T*)gf, gf_stride, side, (T*)Q, (T*)R, kappa, todo, y, dv, stage);
    } else
      hipLaunchKernelGGL((k_reduce_cholqr<T, S>), g, dim3(CQR_THREADS), 0, st, d, na, D, rg, (const S*)site,
                         (const T*)gf, gf_stride, side, (T*)Q, (T*)R, kappa, todo, y);
  }
  // Gram-Schmidt for the items the Cholesky QR left (all items without todo).
  // Real: rows in registers when they fit (up to 2048 rows; measured four
  // times faster at 2048 rows).  Complex: the version that sweeps W in memory
  // (the register version measured slower there: it spills at 1024 rows).
  const long long nrow = (long long)d * na * D * D * D;
  const bool regs = !is_cplx<T>::value && D * rg <= QRR_RMAX && nrow <= 2048;
  if constexpr (!is_cplx<T>::value) {
    if (regs) {
      if (nrow <= 512)
        hipLaunchKernelGGL((k_reduce_qr_reg<T, S, 1, 512>), g, dim3(512), 0, st, d, na, D, rg, (const S*)site,
                           (const T*)gf, gf_stride, side, (T*)Q, (T*)R, kappa, (const int*)todo, y);
      else if (nrow <= 1024)
        hipLaunchKernelGGL((k_reduce_qr_reg<T, S, 2, 512>), g, dim3(512), 0, st, d, na, D, rg, (const S*)site,
                           (const T*)gf, gf_stride, side, (T*)Q, (T*)R, kappa, (const int*)todo, y);
      else
        hipLaunchKernelGGL((k_reduce_qr_reg<T, S, 2, 1024>), g, dim3(1024), 0, st, d, na, D, rg, (const S*)site,
                           (const T*)gf, gf_stride, side, (T*)Q, (T*)R, kappa, (const int*)todo, y);
    }
  }
  if (!regs)
    hipLaunchKernelGGL((k_reduce_qr<T, S>), g, dim3(QR_THREADS), 0, st, d, na, D, rg, (const S*)site, (const T*)gf,
                       gf_stride, side, (T*)Q, (T*)R, kappa, (const int*)todo, y);
}

static hipError_t reduce_dispatch(bool cplx, int site_dtype, int batch, int sides, int d, int na, int D, int rg,
                                  const void* site, const void* gf, long long gf_stride, int side, void* Q, void* R,
                                  const void* site_y, const void* gf_y, void* Q_y, void* R_y, double kappa, int* todo,
                                  hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (!cplx)
    reduce_launch<double, double>(batch, sides, d, na, D, rg, site, gf, gf_stride, side, Q, R, site_y, gf_y, Q_y, R_y,
                                  kappa, todo, st);
  else if (site_dtype == 2)
    reduce_launch<cd, float2>(batch, sides, d, na, D, rg, site, gf, gf_stride, side, Q, R, site_y, gf_y, Q_y, R_y,
                              kappa, todo, st);
  else
    reduce_launch<cd, cd>(batch, sides, d, na, D, rg, site, gf, gf_stride, side, Q, R, site_y, gf_y, Q_y, R_y, kappa,
                          todo, st);
  return hipGetLastError();
}

hipError_t launch_reduce_qr(bool cplx, int site_dtype, int batch, int d, int na, int D, int rg,
                            const void* site, const void* gf, long long gf_stride, int side, void* Q, void* R,
                            double kappa, int* todo, hipStream_t st) {
  return reduce_dispatch(cplx, site_dtype, batch, 1, d, na, D, rg, site, gf, gf_stride, side, Q, R, nullptr, nullptr,
                         nullptr, nullptr, kappa, todo, st);
}

hipError_t launch_reduce_qr_pair(bool cplx, int site_dtype, int batch, int d, int na, int D, int rg,
                                 const void* siteX, const void* gfX, const void* siteY, const void* gfY,
                                 long long gf_stride, void* QX, void* RX, void* QY, void* RY, double kappa, int* todo,
                                 hipStream_t st) {
  return reduce_dispatch(cplx, site_dtype, batch, 2, d, na, D, rg, siteX, gfX, gf_stride, 0, QX, RX, siteY, gfY, QY,
                         RY, kappa, todo, st);
}

// ---------------------------------------------------------------------------
// Recombination: X' = QX MX (new leg r), Y' = QY MY (new leg l).
// rot: 0 = canonical frame, 1 = also rotate back by 90 degrees
// counter-clockwise while writing (vertical bonds).
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_recombine(int p, int D, int R, const T* QX, const T* QY, const T* MX, const T* MY,
                            T* Xn, T* Yn, int rot) {
  const int it = blockIdx.y, side = blockIdx.z;
  const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D3 * D, n = p * D4;
  const T* Qb = (side == 0 ? QX : QY) + (size_t)it * p * D3 * R;
  const T* Mb = (side == 0 ? MX : MY) + (size_t)it * R * D;
  T* Ob = (side == 0 ? Xn : Yn) + (size_t)it * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    // e indexes the canonical-frame output tensor (p, t, l, b, r)
    int r = (int)(e % D), b = (int)((e / D) % D), l = (int)((e / D2) % D), t = (int)((e / D3) % D);
    int pp = (int)(e / D4);
    long long row;
    int c;
    if (side == 0) { row = ((long long)(pp * D + t) * D + l) * D + b; c = r; }
    else { row = ((long long)(pp * D + t) * D + b) * D + r; c = l; }
    T v = zerov<T>();
    for (int a = 0; a < R; ++a) v += Qb[row * R + a] * Mb[a * D + c];
    long long o = e;
    if (rot) {
      // canonical (t, l, b, r) came from original (r', t', l', b') = (t, l, b, r):
      // original[p, t=r, l=t, b=l, r=b]
      o = (long long)pp * D4 + (long long)r * D3 + (long long)t * D2 + (long long)l * D + b;
    }
    Ob[o] = v;
  }
}

hipError_t launch_recombine(bool cplx, int batch, int p, int D, int R, const void* QX, const void* QY,
                            const void* MX, const void* MY, void* Xn, void* Yn, int rot, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  long long n = (long long)p * D * D * D * D;
  int gx = (int)((n + 255) / 256);
  if (gx > 4096) gx = 4096;
  dim3 g(gx, batch, 2), b(256);
  if (cplx)
    hipLaunchKernelGGL(k_recombine<cd>, g, b, 0, st, p, D, R, (const cd*)QX, (const cd*)QY, (const cd*)MX,
                       (const cd*)MY, (cd*)Xn, (cd*)Yn, rot);
  else
    hipLaunchKernelGGL(k_recombine<double>, g, b, 0, st, p, D, R, (const double*)QX, (const double*)QY,
                       (const double*)MX, (const double*)MY, (double*)Xn, (double*)Yn, rot);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rotation by 90 degrees clockwise: new (t, l, b, r) = old (l, b, r, t),
// i.e. new[p, a, b, c, e] = old[p, e, a, b, c].
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_rotate_cw(int p, int D, const T* src, T* dst) {
  const int it = blockIdx.y;
  const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D3 * D, n = p * D4;
  const T* s = src + (size_t)it * n;
  T* o = dst + (size_t)it * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    int ie = (int)(e % D), ic = (int)((e / D) % D), ib = (int)((e / D2) % D), ia = (int)((e / D3) % D);
    int pp = (int)(e / D4);
    o[e] = s[(long long)pp * D4 + (long long)ie * D3 + (long long)ia * D2 + (long long)ib * D + ic];
  }
}

hipError_t launch_rotate_cw(bool cplx, int batch, int p, int D, const void* src, void* dst, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  long long n = (long long)p * D * D * D * D;
  int gx = (int)((n + 255) / 256);
  if (gx > 4096) gx = 4096;
  dim3 g(gx, batch), b(256);
  if (cplx)
    hipLaunchKernelGGL(k_rotate_cw<cd>, g, b, 0, st, p, D, (const cd*)src, (cd*)dst);
  else
    hipLaunchKernelGGL(k_rotate_cw<double>, g, b, 0, st, p, D, (const double*)src, (double*)dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// complex64 storage of site tensors: widen to, or round from, complex128
// ---------------------------------------------------------------------------
__global__ void k_cast_c64(long long n, const void* __restrict__ src, void* __restrict__ dst, int dir) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    if (dir == 0) {
      const float2 v = ((const float2*)src)[e];
      ((double2*)dst)[e] = make_double2((double)v.x, (double)v.y);
    } else {
      const double2 v = ((const double2*)src)[e];
      ((float2*)dst)[e] = make_float2((float)v.x, (float)v.y);
    }
  }
}

hipError_t launch_cast_c64(long long n, const void* src, void* dst, int dir, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int gx = (int)std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_cast_c64, dim3(gx), dim3(256), 0, st, n, src, dst, dir);
  return hipGetLastError();
}

}  // namespace ntu
