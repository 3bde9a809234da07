// Device launchers of the CTMRG expectation values (k_ctm.hip).  Every
// tensor is complex128, dense and row-major; every launcher enqueues on the
// given stream, allocates nothing and does not synchronise.
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace ntu {

constexpr int CTM_MAX_RANK = 8;

// out[i_0 .. i_{r-1}] = op(in[...]) with in's axis perm[k] becoming out's
// axis k: out_shape[k] = in_shape[perm[k]]; op = conj or identity.
hipError_t ctm_permute(const cd* in, cd* out, int rank, const int* in_shape, const int* perm, bool conj,
                       hipStream_t st);
// C (M x N) = A (M x K) B (K x N), row-major; K = 0 writes zeros.  ws
// (ws_el entries, may be null): partial sums when few output tiles meet a
// long K (the K range then split over several workgroups per tile).
hipError_t ctm_gemm(const cd* A, const cd* B, cd* C, int M, int N, int K, cd* ws, long long ws_el, hipStream_t st);
constexpr long long CTM_GEMM_WS = 1ll << 18;  // entries of the partial-sum buffer of a CTMRG object
// A row or column index as digits over n axes (the last fastest): axis a
// has extent dim[a] and moves the address by stride[a] entries.
struct CtmAxes {
  int n = 0;
  int dim[CTM_MAX_RANK] = {};
  long long stride[CTM_MAX_RANK] = {};
};
struct CtmGather {
  CtmAxes ra, ca, rb, cb, rc, cc;  // rows and columns of A, B, C
  int conj_a = 0, conj_b = 0;
};
// C = A B with A (M x K), B (K x N) read and C written through the offsets
// of gd (no permuted copies); K = 0 leaves C untouched.
hipError_t ctm_gemm_gather(const cd* A, const cd* B, cd* C, int M, int N, int K, const CtmGather& gd,
                           hipStream_t st);
// dst[i] = src[i] (real to complex), n entries
hipError_t ctm_widen(const double* src, cd* dst, long long n, hipStream_t st);
// x /= max_i |x_i| (left unchanged when all zero); slot: one unsigned long
// long of scratch
hipError_t ctm_normalise(cd* x, long long n, unsigned long long* slot, hipStream_t st);
// Z (n x k, orthonormal columns) = the left singular vectors of the k
// largest singular values of the n x n matrix rho (n <= CTM_SVD_NMAX), in
// descending order; where rho has numerical rank r < k (singular values at
// most CTM_RANK_EPS sigma_1 beyond), columns r..k-1 are unit vectors e_0,
// e_1, .. in order, each orthogonalised twice against the columns before it
// and kept when more than half its length is left;
// count (<= CTM_SVD_BATCH) independent matrices of one size in one launch.
// ws[b]: CTM_SVD_WS_EXTRA + n^2 entries of scratch when n > CTM_SVD_REG_NMAX
// (else unused).
// One-sided Jacobi on rho's columns: n <= CTM_SVD_REG_NMAX in registers,
// one workgroup per matrix; beyond, in ws, over several workgroups per
// matrix and a chain of launches (the host reads a rotation count back
// between batches of sweeps, so the call waits on the stream).
constexpr int CTM_SVD_NMAX = 1024;
constexpr int CTM_SVD_REG_NMAX = 64;
constexpr int CTM_SVD_BATCH = 4;
constexpr double CTM_RANK_EPS = 1e-12;
constexpr int CTM_SVD_WS_EXTRA = 64;  // entries beyond n^2: rotation counts and a norm
hipError_t ctm_svd_left(int count, const cd* const* rho, int n, int k, cd* const* Z, cd* const* ws, hipStream_t st);
// out[i] = num[i] / den[i], n entries
hipError_t ctm_ratio(const cd* num, const cd* den, cd* out, int n, hipStream_t st);
// out[b] = (sum_t term[b nt + t]) / den[b], nb entries
hipError_t ctm_sum_ratio(const cd* term, const cd* den, cd* out, int nb, int nt, hipStream_t st);
// x[i] = 0, n entries
hipError_t ctm_zero(cd* x, long long n, hipStream_t st);

}  // namespace ntu
