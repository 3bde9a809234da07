// Environment contraction of the nearest-neighbour cluster into the bond
// metric g (Fig. 4): edge double tensors, the two parallel-bond transfers,
// dressed double isometries ("Left", "Right") and the assembly.
//
// Layouts (canonical frame, per item; ' = bra index):
//   EL[x][x'], ER[x][x']                      (D x D)
//   ETX/ETY/EBX/EBY[(u v)][(u' v')]           (D^2 x D^2)
//   EtopT[(T T')][(t t')], EbotT[(c c')][(b b')]
//   QXp[a][b][t][s][l],  QXe = QXp x_l EL      (R D^2 x p D)
//   QYp[B][c][T][s][r],  QYe = QYp x_r ER
//   Left [a][a'][b][b'][t][t']  -> L1[a][a'][T][T'][b][b'] -> L2[a][a'][T][T'][c][c']
//   Right[B][B'][T][T'][c][c']
//   g[(a' B'), (a B)] = sum_{T T' c c'} L2[a a' .] Right[B B' .]
// Every contraction is an "NT" product C(i, j) = sum_k A(i, k) B(j, k) with
// three-level index maps, so no step needs a separate transpose pass.
#include "kernels.h"
#include "mfma_gemm.h"

namespace ntu {

// ---------------------------------------------------------------------------
// generic NT GEMM in FP64 (real or complex), 64 x 64 tiles
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_gemm_nt(const T* __restrict__ A, const T* __restrict__ B,
                                                 T* __restrict__ C, GemmNT d) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN, bt = blockIdx.z;
  const T* Ab = A + idx_off(d.Ab, bt);
  const T* Bb = B + idx_off(d.Bb, bt);
  T* Cb = C + idx_off(d.Cb, bt);
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zerov<T>();
  long long aoff[4], boff[4];
  int arow[4], brow[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int e = tid + u * 256;           // 0 .. 1023 = BM * BK
    arow[u] = e / BK;                // tile row
    int i = i0 + arow[u], j = j0 + arow[u];
    aoff[u] = i < d.M ? idx_off(d.Ai, i) : -1;
    boff[u] = j < d.N ? idx_off(d.Bj, j) : -1;
    brow[u] = arow[u];
  }
  for (int k0 = 0; k0 < d.K; k0 += BK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int e = tid + u * 256, kk = e % BK, k = k0 + kk;
      T va = zerov<T>(), vb = zerov<T>();
      if (k < d.K) {
        long long ko_a = idx_off(d.Ak, k), ko_b = idx_off(d.Bk, k);
        if (aoff[u] >= 0) { va = Ab[aoff[u] + ko_a]; if (d.conjA) va = conjv(va); }
        if (boff[u] >= 0) { vb = Bb[boff[u] + ko_b]; if (d.conjB) vb = conjv(vb); }
      }
      As[kk][arow[u]] = va;
      Bs[kk][brow[u]] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { a[u] = As[kk][ty + 16 * u]; b[u] = Bs[kk][tx + 16 * u]; }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int i = i0 + ty + 16 * u;
    if (i >= d.M) continue;
    long long ci = idx_off(d.Ci, i);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int j = j0 + tx + 16 * v;
      if (j >= d.N) continue;
      Cb[ci + idx_off(d.Cj, j)] = acc[u][v];
    }
  }
}

static hipError_t gemm_nt(bool cplx, const void* A, const void* B, void* C, const GemmNT& d, hipStream_t st) {
  dim3 g((d.N + 63) / 64, (d.M + 63) / 64, d.batch), b(256);
  if (cplx)
    hipLaunchKernelGGL(k_gemm_nt<cd>, g, b, 0, st, (const cd*)A, (const cd*)B, (cd*)C, d);
  else
    hipLaunchKernelGGL(k_gemm_nt<double>, g, b, 0, st, (const double*)A, (const double*)B, (double*)C, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small products of the environment (edge double tensors and the two
// parallel-bond transfers), M, N <= 64: C(i, j) = sum_k A(i, k) op(B(j, k)),
// op = conj or identity, several products per launch (blockIdx.x selects the
// product, blockIdx.y the item).  K is staged through shared memory in
// chunks, loaded with the fastest-varying index of each operand's memory
// layout on consecutive threads, from offset tables built once per chunk.
// M, N > 16: 4 x 4 outputs per thread over a 64 x 64 tile.  M, N <= 16 (the
// D x D edges with long K): each output is summed by 256 / (M N) threads over
// interleaved k and the parts meet in shared memory.
// ---------------------------------------------------------------------------
struct SmallNT {
  const void* A;
  const void* B;
  void* C;
  long long sa, sb, sc;  // item strides (elements)
  Idx3 Ai, Ak, Bj, Bk;   // row / contraction maps
  long long ldc;         // C row stride
  int M, N, K;
  int conjB;
  int a_kfast, b_kfast;  // 1: consecutive k are adjacent in memory
};
struct SmallBatch {
  SmallNT p[8];
};
constexpr int SM_T = 64, SM_KC = 32, SM_KCS = 128;

template <class T>
__global__ void __launch_bounds__(256) k_small_nt(SmallBatch sb) {
  const SmallNT& d = sb.p[blockIdx.x];
  const int it = blockIdx.y, tid = threadIdx.x;
  const T* A = (const T*)d.A + (size_t)it * d.sa;
  const T* B = (const T*)d.B + (size_t)it * d.sb;
  T* C = (T*)d.C + (size_t)it * d.sc;
  const int M = d.M, N = d.N, K = d.K;
  const bool small = M <= 16 && N <= 16;
  const int KC = small ? SM_KCS : SM_KC;
  __shared__ T SA[SM_KCS * 17 > SM_KC * (SM_T + 1) ? SM_KCS * 17 : SM_KC * (SM_T + 1)];
  __shared__ T SB[SM_KCS * 17 > SM_KC * (SM_T + 1) ? SM_KCS * 17 : SM_KC * (SM_T + 1)];
  __shared__ long long roA[SM_T], roB[SM_T];
  __shared__ long long koA[SM_KCS], koB[SM_KCS];
  __shared__ T part[256];
  const int lda = small ? 17 : SM_T + 1;  // S[k * lda + i]
  for (int i = tid; i < SM_T; i += 256) {
    roA[i] = i < M ? idx_off(d.Ai, i) : 0;
    roB[i] = i < N ? idx_off(d.Bj, i) : 0;
  }
  const int ty = tid >> 4, tx = tid & 15;
  T acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = zerov<T>();
  const int mn = M * N, kpar = small ? 256 / (mn > 0 ? mn : 1) : 1;
  const int si = small ? tid % (mn > 0 ? mn : 1) / N : 0, sj = small ? tid % (mn > 0 ? mn : 1) % N : 0;
  const int skp = small ? tid / (mn > 0 ? mn : 1) : 0;
  T sacc = zerov<T>();
  for (int k0 = 0; k0 < K; k0 += KC) {
    const int kc = min(KC, K - k0);
    __syncthreads();  // previous chunk consumed
    for (int k = tid; k < kc; k += 256) {
      koA[k] = idx_off(d.Ak, k0 + k);
      koB[k] = idx_off(d.Bk, k0 + k);
    }
    __syncthreads();
    // stage A (M x kc) and B (N x kc) as S[k][i]
    for (int e = tid; e < M * kc; e += 256) {
      const int i = d.a_kfast ? e / kc : e % M, k = d.a_kfast ? e % kc : e / M;
      SA[k * lda + i] = A[roA[i] + koA[k]];
    }
    for (int e = tid; e < N * kc; e += 256) {
      const int j = d.b_kfast ? e / kc : e % N, k = d.b_kfast ? e % kc : e / N;
      const T v = B[roB[j] + koB[k]];
      SB[k * lda + j] = d.conjB ? conjv(v) : v;
    }
    __syncthreads();
    if (small) {
      if (skp < kpar && tid < kpar * mn)
        for (int k = skp; k < kc; k += kpar) sacc += SA[k * lda + si] * SB[k * lda + sj];
    } else {
      for (int k = 0; k < kc; ++k) {
        T a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = SA[k * lda + ty + 16 * u];
          b[u] = SB[k * lda + tx + 16 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
      }
    }
  }
  if (small) {
    __syncthreads();
    part[tid] = sacc;
    __syncthreads();
    if (tid < mn) {
      T s = zerov<T>();
      for (int q = 0; q < kpar; ++q) s += part[q * mn + tid];
      C[(size_t)(tid / N) * d.ldc + tid % N] = s;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = ty + 16 * u;
      if (i >= M) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = tx + 16 * v;
        if (j < N) C[(size_t)i * d.ldc + j] = acc[u][v];
      }
    }
  }
}

static hipError_t small_nt(bool cplx, const SmallBatch& b, int np, int batch, hipStream_t st) {
  dim3 g(np, batch), bl(256);
  if (cplx) hipLaunchKernelGGL(k_small_nt<cd>, g, bl, 0, st, b);
  else hipLaunchKernelGGL(k_small_nt<double>, g, bl, 0, st, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// QXp / QXe (and QYp / QYe): regroup the isometry rows so that the legs
// contracted in the half environments come last, and multiply the leg that
// meets L (or Rn) by EL (or ER).
//   X side: Q rows (s, t, l, b)  -> out[a][b][t][s][l]
//   Y side: Q rows (s, t, b, r)  -> out[B][c=b][T=t][s][r]
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_qprep(int p, int D, int R, int side, const T* __restrict__ Q, const T* __restrict__ E,
                        long long e_stride, T* __restrict__ Qp, T* __restrict__ Qe, long long out_stride) {
  const int it = blockIdx.y;
  const long long D2 = (long long)D * D, D3 = D2 * D;
  const long long n = (long long)R * D2 * p * D;
  const T* Qi = Q + (size_t)it * p * D3 * R;
  const T* Ei = E + (size_t)it * e_stride;
  T* Op = Qp + (size_t)it * out_stride;
  T* Oe = Qe + (size_t)it * out_stride;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    int x = (int)(e % D);                  // l (X) or r (Y): leg that meets the edge tensor
    int s = (int)((e / D) % p);
    int t = (int)((e / (D * p)) % D);
    int b = (int)((e / (D2 * p)) % D);
    int a = (int)(e / (D3 * p));
    // row of Q holding (s, t, b, x)
    long long rbase = side == 0 ? (long long)s * D3 + (long long)t * D2 + b          // + x * D
                                : (long long)s * D3 + (long long)t * D2 + (long long)b * D;  // + x
    long long xs = side == 0 ? D : 1;
    Op[e] = Qi[(rbase + x * xs) * R + a];
    T acc = zerov<T>();
    for (int y = 0; y < D; ++y) acc += Qi[(rbase + y * xs) * R + a] * Ei[y * D + x];
    Oe[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// Half environments (Fig. 4(c)) with the short contraction K = p D:
//   Left[(a b t), (a' b' t')]  = sum_s QXe[(a b t), s] conj(QXp[(a' b' t'), s]),
//     stored Left[a][a'][b][b'][t][t'];
//   Right[(B c T), (B' c' T')] = sum_s QYe[(B c T), s] conj(QYp[(B' c' T'), s]),
//     stored Right[B][B'][T][T'][c][c'].
// The product is bound by its output writes, so it runs on the vector units:
// one block per (item, a, a') holds the bra rows of a' in shared memory
// (padded rows), loops over the ket index b (X) or T (Y), and consecutive
// threads write consecutive output elements.  TO: output scalar (float for
// the split-precision paths, double for the FP64 path); complex outputs are
// (re, im) pairs.
// ---------------------------------------------------------------------------
template <class T, class TO>
__global__ void __launch_bounds__(256) k_half_env(int p, int D, int R, int side, const T* __restrict__ Qe,
                                                  const T* __restrict__ Qp, long long qstride, TO* __restrict__ out,
                                                  long long ostride) {
  extern __shared__ double shmem[];
  constexpr int CW = is_cplx<T>::value ? 2 : 1;
  const int pD = p * D, ld = pD + 1, D2 = D * D, D3 = D2 * D;
  const long long D4 = (long long)D2 * D2;
  const int RR = R * R;
  const int it = blockIdx.x / RR, a = (blockIdx.x / R) % R, ap = blockIdx.x % R;
  const int tid = threadIdx.x;
  T* P = (T*)shmem;        // D2 bra rows of ap, padded
  T* L = P + D2 * ld;      // D ket rows of the current b (X) or T (Y)
  const T* Qei = Qe + (size_t)it * qstride;
  const T* Qpi = Qp + (size_t)it * qstride;
  TO* O = out + (size_t)it * ostride * CW;
  // bra rows: X: (b', t') at P[b' D + t'];  Y: (c', T') at P[T' D + c']
  for (int e = tid; e < D2 * pD; e += blockDim.x) {
    const int r = e / pD, sg = e % pD;
    const int slot = side == 0 ? r : (r % D) * D + r / D;
    P[slot * ld + sg] = Qpi[((size_t)ap * D2 + r) * pD + sg];
  }
  for (int kb = 0; kb < D; ++kb) {
    __syncthreads();
    // ket rows: X: (a, kb, t) for t < D;  Y: (a, c, kb) for c < D
    for (int e = tid; e < D * pD; e += blockDim.x) {
      const int u = e / pD, sg = e % pD;
      const size_t row = side == 0 ? ((size_t)a * D + kb) * D + u : ((size_t)a * D + u) * D + kb;
      L[u * ld + sg] = Qei[row * pD + sg];
    }
    __syncthreads();
    const size_t obase = (size_t)a * R * D4 + (size_t)ap * D4 + (size_t)kb * D3;
    for (int e = tid; e < D3; e += blockDim.x) {
      // X: e = (b', t, t'), ket row t, bra slot b' D + t'
      // Y: e = (T', c, c'), ket row c, bra slot T' D + c'
      const int hi = e / D2, mid = (e / D) % D, lo = e % D;
      const int ku = mid, ps = hi * D + lo;
      T acc = zerov<T>();
      for (int sg = 0; sg < pD; ++sg) acc += mulc(L[ku * ld + sg], P[ps * ld + sg]);
      if constexpr (CW == 2) {
        O[2 * (obase + e)] = (TO)rev(acc);
        O[2 * (obase + e) + 1] = (TO)imv(acc);
      } else {
        O[obase + e] = (TO)rev(acc);
      }
    }
  }
}

static size_t half_env_shmem(bool cplx, int p, int D) {
  return (size_t)(D * D + D) * (p * D + 1) * (cplx ? 16 : 8);
}

// Left into H0 and Right into H2 (FP64 path)
static hipError_t half_env(bool cplx, int batch, int p, int D, int R, const void* QXe, const void* QXp,
                           const void* QYe, const void* QYp, long long qs, void* H0, void* H2, long long hs,
                           hipStream_t st) {
  const size_t shm = half_env_shmem(cplx, p, D);
  dim3 g(batch * R * R), b(256);
  for (int side = 0; side < 2; ++side) {
    const void* Qe = side == 0 ? QXe : QYe;
    const void* Qp = side == 0 ? QXp : QYp;
    void* O = side == 0 ? H0 : H2;
    if (cplx)
      hipLaunchKernelGGL((k_half_env<cd, double>), g, b, shm, st, p, D, R, side, (const cd*)Qe, (const cd*)Qp, qs,
                         (double*)O, hs);
    else
      hipLaunchKernelGGL((k_half_env<double, double>), g, b, shm, st, p, D, R, side, (const double*)Qe,
                         (const double*)Qp, qs, (double*)O, hs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

EnvSizes env_sizes(int p, int D, int R) {
  EnvSizes s;
  long long D2 = (long long)D * D, D4 = D2 * D2;
  s.p = p; s.D = D; s.R = R;
  s.e_small = 2 * D2 + 6 * D4;
  s.qp = (long long)R * D2 * p * D;
  s.half = (long long)R * R * D4;
  return s;
}

// element size of the large intermediates: the compute type on the FP64 path,
// float (real) / float2 (complex) on the mixed paths
static size_t half_elem(bool cplx, int precision) {
  if (precision == 0) return cplx ? 16 : 8;
  return cplx ? 8 : 4;
}

bool env_precision_supported(bool cplx, int precision, int D) {
  if (precision == NTU_PREC_F64 || precision == NTU_PREC_BF16X3 || precision == NTU_PREC_BF16X6) return true;
  // FP16X3 scales each operand block by block inside the fused kernels:
  // complex metrics with D^2 <= 64 (the fused path)
  return precision == NTU_PREC_FP16X3 && e45_supported(cplx, precision, D);
}

size_t env_workspace_bytes(bool cplx, int precision, int batch, int p, int D, int R) {
  EnvSizes s = env_sizes(p, D, R);
  size_t el = cplx ? 16 : 8;
  size_t per = (size_t)(s.e_small + 4 * s.qp) * el + 3 * (size_t)s.half * half_elem(cplx, precision);
  size_t extra = precision == 0 ? 0 : mixed_partial_bytes(cplx, batch, R, D);
  return per * (size_t)batch + extra + 4096;
}

hipError_t launch_env_contract(bool cplx, int precision, int batch, int p, int D, int R, const void* QX,
                               const void* QY, const void* const nbr[6], void* g, void* ws, size_t ws_bytes,
                               hipStream_t st, const ProfHook& ph, int part, int e6_ks) {
  if (batch <= 0) return hipSuccess;
  if (env_workspace_bytes(cplx, precision, batch, p, D, R) > ws_bytes) return hipErrorOutOfMemory;
  const EnvSizes s = env_sizes(p, D, R);
  const size_t el = cplx ? 16 : 8, hel = half_elem(cplx, precision);
  const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D2 * D2;
  const long long site = p * D4;
  // carve the workspace: small (compute type) part for all items, then the big buffers
  char* w = (char*)ws;
  char* EL = w;                          // per item e_small elements
  char* ER = EL + D2 * el;
  char* ETX = ER + D2 * el;
  char* ETY = ETX + D4 * el;
  char* EBX = ETY + D4 * el;
  char* EBY = EBX + D4 * el;
  char* ETT = EBY + D4 * el;             // EtopT
  char* EBT = ETT + D4 * el;             // EbotT
  const long long es = s.e_small;        // item stride of the small block (elements)
  char* QXp = w + (size_t)batch * es * el;
  char* QXe = QXp + (size_t)batch * s.qp * el;
  char* QYp = QXe + (size_t)batch * s.qp * el;
  char* QYe = QYp + (size_t)batch * s.qp * el;
  char* H0 = QYe + (size_t)batch * s.qp * el;          // Left, later L2
  char* H1 = H0 + (size_t)batch * s.half * hel;        // L1
  char* H2 = H1 + (size_t)batch * s.half * hel;        // Right
  hipError_t err;
#define NTU_TRY(x) do { err = (x); if (err != hipSuccess) return err; } while (0)

  // 1. edge double tensors (Fig. 4(a,b)): E(i, j) = sum_k T(i, k) conj(T(j, k)),
  //    and 2. the parallel-bond transfers
  //    EtopT[(T T')][(t t')] = sum_{v v'} ETY[T v T' v'] ETX[t v t' v'] (EbotT alike)
  if (part != 2) {
  ph(PK_EDGES, 0);
  if (D2 <= SM_T) {
    SmallBatch eb{};
    auto gram = [&](int slot, const void* Tn, char* out, Idx3 Ii, Idx3 Ik, int M, int K, int kfast) {
      SmallNT& q = eb.p[slot];
      q.A = Tn; q.B = Tn; q.C = out;
      q.sa = site; q.sb = site; q.sc = es;
      q.Ai = Ii; q.Ak = Ik; q.Bj = Ii; q.Bk = Ik;
      q.ldc = M; q.M = M; q.N = M; q.K = K; q.conjB = 1;
      q.a_kfast = kfast; q.b_kfast = kfast;
    };
    gram(0, nbr[0], EL, idx1(1), idx1(D), D, (int)(p * D3), 0);                                 // k = (p, t, l, b)
    gram(1, nbr[5], ER, idx1(D2), idx2((int)D2, D3, 1), D, (int)(p * D3), 1);                   // k = ((p, t), (b, r))
    gram(2, nbr[1], ETX, idx1(1), idx1(D2), (int)D2, (int)(p * D2), 0);                          // u = b, v = r
    gram(3, nbr[3], ETY, idx2(D, D, D2), idx2(D, D3, 1), (int)D2, (int)(p * D2), 1);             // u = b, v = l
    gram(4, nbr[2], EBX, idx2(D, D3, 1), idx2((int)D2, D4, D), (int)D2, (int)(p * D2), 0);       // u = t, v = r
    gram(5, nbr[4], EBY, idx2(D, D3, D2), idx2((int)D2, D4, 1), (int)D2, (int)(p * D2), 1);      // u = t, v = l
    NTU_TRY(small_nt(cplx, eb, 6, batch, st));
    SmallBatch tb{};
    auto transfer = [&](int slot, const char* Ay, const char* Bx, char* out) {
      SmallNT& q = tb.p[slot];
      q.A = Ay; q.B = Bx; q.C = out;
      q.sa = es; q.sb = es; q.sc = es;
      q.Ai = idx2(D, D3, D); q.Ak = idx2(D, D2, 1);
      q.Bj = idx2(D, D3, D); q.Bk = idx2(D, D2, 1);
      q.ldc = D2; q.M = (int)D2; q.N = (int)D2; q.K = (int)D2; q.conjB = 0;
      q.a_kfast = 1; q.b_kfast = 1;
    };
    transfer(0, ETY, ETX, ETT);
    transfer(1, EBY, EBX, EBT);
    NTU_TRY(small_nt(cplx, tb, 2, batch, st));
  } else {
  auto edge2 = [&](const void* T, char* out, Idx3 Ii, Idx3 Ik, int M, int K) {
    GemmNT d{};
    d.M = M; d.N = M; d.K = K; d.batch = batch;
    d.Ab = idx1(site); d.Bb = idx1(site); d.Cb = idx1(es);
    d.Ai = Ii; d.Ak = Ik; d.Bj = Ii; d.Bk = Ik;
    d.Ci = idx1(M); d.Cj = idx1(1);
    d.conjA = 0; d.conjB = 1;
    return gemm_nt(cplx, T, T, out, d, st);
  };
  NTU_TRY(edge2(nbr[0], EL, idx1(1), idx1(D), D, (int)(p * D3)));
  NTU_TRY(edge2(nbr[5], ER, idx1(D2), idx2((int)D2, D3, 1), D, (int)(p * D3)));
  NTU_TRY(edge2(nbr[1], ETX, idx1(1), idx1(D2), (int)D2, (int)(p * D2)));
  NTU_TRY(edge2(nbr[3], ETY, idx2(D, D, D2), idx2(D, D3, 1), (int)D2, (int)(p * D2)));
  NTU_TRY(edge2(nbr[2], EBX, idx2(D, D3, 1), idx2((int)D2, D4, D), (int)D2, (int)(p * D2)));
  NTU_TRY(edge2(nbr[4], EBY, idx2(D, D3, D2), idx2((int)D2, D4, 1), (int)D2, (int)(p * D2)));
  GemmNT d{};
  d.M = (int)D2; d.N = (int)D2; d.K = (int)D2; d.batch = batch;
  d.Ab = idx1(es); d.Bb = idx1(es); d.Cb = idx1(es);
  d.Ai = idx2(D, D3, D); d.Ak = idx2(D, D2, 1);
  d.Bj = idx2(D, D3, D); d.Bk = idx2(D, D2, 1);
  d.Ci = idx1(D2); d.Cj = idx1(1);
  NTU_TRY(gemm_nt(cplx, ETY, ETX, ETT, d, st));
  NTU_TRY(gemm_nt(cplx, EBY, EBX, EBT, d, st));
  }
  ph(PK_EDGES, 1);
  }
  if (part == 1) return hipSuccess;

  // 3. regrouped isometries dressed with EL / ER
  ph(PK_QPREP, 0);
  {
    long long n = s.qp;
    int gx = (int)((n + 255) / 256);
    if (gx > 2048) gx = 2048;
    dim3 gg(gx, batch), bb(256);
    if (cplx) {
      hipLaunchKernelGGL(k_qprep<cd>, gg, bb, 0, st, p, D, R, 0, (const cd*)QX, (const cd*)EL, es, (cd*)QXp, (cd*)QXe, s.qp);
      hipLaunchKernelGGL(k_qprep<cd>, gg, bb, 0, st, p, D, R, 1, (const cd*)QY, (const cd*)ER, es, (cd*)QYp, (cd*)QYe, s.qp);
    } else {
      hipLaunchKernelGGL(k_qprep<double>, gg, bb, 0, st, p, D, R, 0, (const double*)QX, (const double*)EL, es, (double*)QXp, (double*)QXe, s.qp);
      hipLaunchKernelGGL(k_qprep<double>, gg, bb, 0, st, p, D, R, 1, (const double*)QY, (const double*)ER, es, (double*)QYp, (double*)QYe, s.qp);
    }
    NTU_TRY(hipGetLastError());
  }
  ph(PK_QPREP, 1);

  const int pD = p * D;
  const long long RD4 = (long long)R * D4;
  if (precision == 0) {
    // 4. Left[a][a'][b][b'][t][t'] = sum_{s l'} QXe[(a b t)][(s l')] conj(QXp[(a' b' t')][(s l')])
    GemmNT d{};
    d.M = (int)(R * D2); d.N = (int)(R * D2); d.K = pD; d.batch = batch;
    d.Ab = idx1(s.qp); d.Bb = idx1(s.qp); d.Cb = idx1(s.half);
    d.Ai = idx1(pD); d.Ak = idx1(1); d.Bj = idx1(pD); d.Bk = idx1(1);
    d.conjB = 1;
    d.Ci = idx3(D, D, RD4, D3, D); d.Cj = idx3(D, D, D4, D2, 1);
    ph(PK_LEFTRIGHT, 0);
    if (half_env_shmem(cplx, p, D) <= 64 * 1024) {
      NTU_TRY(half_env(cplx, batch, p, D, R, QXe, QXp, QYe, QYp, s.qp, H0, H2, s.half, st));
    } else {
      NTU_TRY(gemm_nt(cplx, QXe, QXp, H0, d, st));
      // Right[B][B'][T][T'][c][c'] from rows (B, c, T)
      d.Ci = idx3(D, D, RD4, D, D3); d.Cj = idx3(D, D, D4, 1, D2);
      NTU_TRY(gemm_nt(cplx, QYe, QYp, H2, d, st));
    }
    ph(PK_LEFTRIGHT, 1);
    // 5. L1[a a'][T T'][b b'] = sum_{t t'} Left[(a a' b b')][(t t')] EtopT[(T T')][(t t')]
    GemmNT e{};
    e.M = (int)(R * R * D2); e.N = (int)D2; e.K = (int)D2; e.batch = batch;
    e.Ab = idx1(s.half); e.Bb = idx1(es); e.Cb = idx1(s.half);
    e.Ai = idx1(D2); e.Ak = idx1(1); e.Bj = idx1(D2); e.Bk = idx1(1);
    e.Ci = idx2((int)D2, D4, 1); e.Cj = idx1(D2);
    ph(PK_E4, 0);
    NTU_TRY(gemm_nt(cplx, H0, ETT, H1, e, st));
    ph(PK_E4, 1);
    // 6. L2[(a a' T T')][(c c')] = sum_{b b'} L1[(a a' T T')][(b b')] EbotT[(c c')][(b b')]
    e.Ci = idx1(D2); e.Cj = idx1(1);
    ph(PK_E5, 0);
    NTU_TRY(gemm_nt(cplx, H1, EBT, H0, e, st));
    ph(PK_E5, 1);
    // 7. g[(a' B'), (a B)] = sum_K L2[(a a')][K] Right[(B B')][K]
    GemmNT f{};
    f.M = R * R; f.N = R * R; f.K = (int)D4; f.batch = batch;
    f.Ab = idx1(s.half); f.Bb = idx1(s.half); f.Cb = idx1((long long)R * R * R * R);
    f.Ai = idx1(D4); f.Ak = idx1(1); f.Bj = idx1(D4); f.Bk = idx1(1);
    f.Ci = idx2(R, R, (long long)R * R * R); f.Cj = idx2(R, 1, (long long)R * R);
    ph(PK_E6, 0);
    NTU_TRY(gemm_nt(cplx, H0, H2, g, f, st));
    ph(PK_E6, 1);
  } else {
    // the products of steps 4-7 on the matrix cores in split precision
    NTU_TRY(launch_env_heavy_mixed(cplx, precision, batch, p, D, R, QXe, QXp, QYe, QYp, ETT, EBT, es, s.qp,
                                   s.half, H0, H1, H2, g, st, ph, e6_ks));
  }
#undef NTU_TRY
  return hipSuccess;
}

}  // namespace ntu
