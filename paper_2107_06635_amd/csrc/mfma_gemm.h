// Descriptors of the NT products C(i, j) = sum_k A(i, k) B(j, k) used by the
// environment contraction, and the split-precision MFMA path.
#pragma once
#include <algorithm>
#include "common.h"
#include "ntu.h"
#include "kernels.h"

namespace ntu {

struct GemmNT {
  int M, N, K, batch;
  Idx3 Ab, Ai, Ak;   // A: item offset, row i, column k
  Idx3 Bb, Bj, Bk;   // B: item offset, row j, column k
  Idx3 Cb, Ci, Cj;   // C: item offset, row i, column j
  int conjA, conjB;
};

// Left/Right, L1, L2 and g of the environment contraction in split precision
// (BF16x3, FP16x3 or BF16x6 on MFMA with FP32 accumulation).  Inputs QXe,
// QXp, QYe, QYp, EtopT, EbotT are in the compute type; H0, H1, H2 hold the
// FP32 intermediates; g is written in the compute type.
hipError_t launch_env_heavy_mixed(bool cplx, int precision, int batch, int p, int D, int R, const void* QXe,
                                  const void* QXp, const void* QYe, const void* QYp, const void* ETT,
                                  const void* EBT, long long es, long long qs, long long hs, void* H0, void* H1,
                                  void* H2, void* g, hipStream_t st, const struct ProfHook& ph, int e6_ks = 0);

// Environment products fused per (item, a, a') block on the matrix cores
// (complex, BF16x3 or BF16x6, D^2 <= 64): Right into H2, L2 (from Left, L1
// formed and consumed in shared memory) into H0; H1 holds the prepared
// EtopT / EbotT operands (e45_frag_bytes).  Item stride hs complex elements.
bool e45_supported(bool cplx, int precision, int D);
size_t e45_frag_bytes(int precision, int batch, int D);
// FP16X3 scales (float, in H1 after the fragments): e[item][2] of EtopT /
// EbotT; left[item][R^2], right[item][R^2]: the power-of-two factor each row
// of the L2 / Right pieces carries
struct E45Scales {
  float* e;
  float* left;
  float* right;
  float* blk;  // per item the scales of the isometry blocks QXe[a], QXp[a], QYe[b], QYp[b] (4 R)
};
E45Scales e45_scales(void* H1, int precision, int batch, int D, int R);
size_t e45_scale_bytes(int batch, int R);
hipError_t launch_env_fused(int precision, int batch, int p, int D, int R, const void* QXe, const void* QXp,
                            const void* QYe, const void* QYp, const void* ETT, const void* EBT, long long es,
                            long long qs, void* H0, void* H1, void* H2, long long hs, hipStream_t st,
                            const struct ProfHook& ph);

// K split of the final assembly g = L2 Right^T (E6): e6_ks > 0 asks for that
// many K chunks (autotuning), at most e6_ksplit_max; 0 takes the heuristic
// e6_ksplit_default.  The workspace reserves the partial sums of the largest.
constexpr int E6_KS_TUNE_MAX = 4;
int e6_ksplit_default(bool cplx, int batch, int R, int D);
int e6_ksplit_max(bool cplx, int batch, int R, int D);
// bytes of FP64 split-K partial sums the final assembly needs after H2
size_t mixed_partial_bytes(bool cplx, int batch, int R, int D);

}  // namespace ntu
