// Gate split (Fig. 2(a)), reduction + QR (Fig. 2(b)), recombination
// (Fig. 2(e)) and the 90-degree rotation of site tensors.
#include "kernels.h"
#include "linalg.h"

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
// Reduction: W = gate factor applied to the site tensor, then Gram-Schmidt QR
// with the projection applied twice and the rank rule.  One workgroup per item.
// ---------------------------------------------------------------------------
template <class T> NTU_DEV T load_site(const double* p, long long i) { return realv<T>(p[i]); }
template <class T> NTU_DEV T load_site(const cd* p, long long i);
template <> NTU_DEV cd load_site<cd>(const cd* p, long long i) { return p[i]; }
template <class T> NTU_DEV T load_site(const float2* p, long long i);
template <> NTU_DEV cd load_site<cd>(const float2* p, long long i) {
  float2 v = p[i];
  return cd{(double)v.x, (double)v.y};
}

constexpr int QR_THREADS = 256;
constexpr int QR_RMAX = 32;

template <class T, class S>
__global__ void __launch_bounds__(QR_THREADS) k_reduce_qr(int d, int na, int D, int rg, const S* site,
                                                         const T* gf, long long gf_stride, int side, T* Q, T* Rm,
                                                         double kappa) {
  __shared__ double red[16 * 64];
  __shared__ double hv[2 * QR_RMAX];
  __shared__ double cacc[2 * QR_RMAX];
  constexpr int NC = is_cplx<T>::value ? 2 : 1;
  const int it = blockIdx.x, tid = threadIdx.x;
  const int p = d * na, R = D * rg;
  const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D3 * D;
  const long long nrow = p * D3;
  const S* X = site + (size_t)it * p * D4;
  const T* G = gf + (size_t)it * gf_stride;
  T* Qi = Q + (size_t)it * nrow * R;
  T* Ri = Rm + (size_t)it * R * R;

  // 1. W into Q (row-major nrow x R)
  for (long long e = tid; e < nrow * R; e += blockDim.x) {
    long long row = e / R;
    int col = (int)(e % R), q = col / rg, k = col % rg;
    int i4 = (int)(row % D), i3 = (int)((row / D) % D), t = (int)((row / D2) % D);
    int pa = (int)(row / D3), sp = pa / na, a = pa % na;
    T v = zerov<T>();
    for (int s = 0; s < d; ++s) {
      long long base = (long long)(s * na + a) * D4 + t * D3;
      // X side: rows (s',a,t,l=i3,b=i4), bond = r = q ; Y side: rows (s',a,t,b=i3,r=i4), bond = l = q
      long long off = side == 0 ? base + i3 * D2 + i4 * D + q : base + q * D2 + i3 * D + i4;
      v += G[(sp * d + s) * rg + k] * load_site<T>(X, off);
    }
    Qi[e] = v;
  }
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

hipError_t launch_reduce_qr(bool cplx, int site_dtype, int batch, int d, int na, int D, int rg,
                            const void* site, const void* gf, long long gf_stride, int side, void* Q, void* R,
                            double kappa, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  dim3 g(batch), b(QR_THREADS);
  if (!cplx) {
    hipLaunchKernelGGL((k_reduce_qr<double, double>), g, b, 0, st, d, na, D, rg, (const double*)site,
                       (const double*)gf, gf_stride, side, (double*)Q, (double*)R, kappa);
  } else if (site_dtype == 2) {
    hipLaunchKernelGGL((k_reduce_qr<cd, float2>), g, b, 0, st, d, na, D, rg, (const float2*)site,
                       (const cd*)gf, gf_stride, side, (cd*)Q, (cd*)R, kappa);
  } else {
    hipLaunchKernelGGL((k_reduce_qr<cd, cd>), g, b, 0, st, d, na, D, rg, (const cd*)site, (const cd*)gf,
                       gf_stride, side, (cd*)Q, (cd*)R, kappa);
  }
  return hipGetLastError();
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

}  // namespace ntu
