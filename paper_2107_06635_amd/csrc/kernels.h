// Host-side launchers of the libntu kernels.  Every launcher enqueues on the
// given stream and returns the launch status; none allocates or synchronises.
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace ntu {

// message returned by ntu_last_error(NULL) (calls without a context)
void set_global_error(const char* msg);

// Kernel classes timed by the optional event profiler of a context.
enum ProfKind {
  PK_ROTATE = 0, PK_GATE, PK_REDUCE, PK_EDGES, PK_QPREP, PK_LEFTRIGHT, PK_E4, PK_E5, PK_E6, PK_E6RED,
  PK_HERM, PK_CLIP, PK_FIT, PK_RECOMB, PK_CERT, PK_COUNT
};
// mark(ctx, kind, 0) before and mark(ctx, kind, 1) after a launch (nullable)
struct ProfHook {
  void (*mark)(void* ctx, int kind, int phase);
  void* ctx;
  void operator()(int kind, int phase) const {
    if (mark) mark(ctx, kind, phase);
  }
};

hipError_t launch_superop(bool cplx_gate, int batch, const void* gate, double* S, hipStream_t st);
hipError_t launch_gate_split(bool cplx, int batch, int d, int rg, const void* gate, void* GA, void* GB,
                             double* sigma, hipStream_t st);
hipError_t launch_reduce_qr(bool cplx, int site_dtype, int batch, int d, int na, int D, int rg,
                            const void* site, const void* gf, long long gf_stride, int side, void* Q, void* R,
                            double kappa, int* todo, hipStream_t st);
// both sides of a bond in one launch (X: side 0, Y: side 1); todo: 2 batch ints
hipError_t launch_reduce_qr_pair(bool cplx, int site_dtype, int batch, int d, int na, int D, int rg,
                                 const void* siteX, const void* gfX, const void* siteY, const void* gfY,
                                 long long gf_stride, void* QX, void* RX, void* QY, void* RY, double kappa, int* todo,
                                 hipStream_t st);
hipError_t launch_recombine(bool cplx, int batch, int p, int D, int R, const void* QX, const void* QY,
                            const void* MX, const void* MY, void* Xn, void* Yn, int rot, hipStream_t st);
hipError_t launch_rotate_cw(bool cplx, int batch, int p, int D, const void* src, void* dst, hipStream_t st);
// complex64 <-> complex128 copy of n elements: dir 0 widens src (complex64)
// into dst (complex128), dir 1 rounds src (complex128) into dst (complex64)
hipError_t launch_cast_c64(long long n, const void* src, void* dst, int dir, hipStream_t st);

// ---------------------------------------------------------------------------
// environment contraction
// ---------------------------------------------------------------------------
// Workspace layout of one environment contraction (per item, in elements of
// the compute type unless noted).
struct EnvSizes {
  int p, D, R;
  long long e_small;   // EL, ER (D^2 each) + 4 edge tensors (D^4 each) + Etop^T, Ebot^T (D^4 each)
  long long qp;        // QXp / QXe / QYp / QYe: R D^2 p D each
  long long half;      // Left / Right / L1 / L2: R^2 D^4 each
};
EnvSizes env_sizes(int p, int D, int R);
// whether ntu_env_contract implements this precision for the compute type and D
bool env_precision_supported(bool cplx, int precision, int D);
// bytes of workspace needed for `batch` items at this shape and precision
size_t env_workspace_bytes(bool cplx, int precision, int batch, int p, int D, int R);
// part 0: the whole contraction; 1: only the edge tensors and transfers
// (steps 1-2, they read only the neighbours); 2: the rest (they must have run)
hipError_t launch_env_contract(bool cplx, int precision, int batch, int p, int D, int R, const void* QX,
                               const void* QY, const void* const nbr[6], void* g, void* ws, size_t ws_bytes,
                               hipStream_t st, const ProfHook& ph, int part = 0, int e6_ks = 0);

// ---------------------------------------------------------------------------
// metric repair and fit
// ---------------------------------------------------------------------------
size_t fix_workspace_bytes(bool cplx, int batch, int n);
// shift_rel > 0: also test g - shift_rel ||g||_F I and report per item in
// cert (1 = certified, may be NULL)
hipError_t launch_metric_fix(bool cplx, int batch, int n, void* g, int mode, double* stats, int stats_stride,
                             void* ws, hipStream_t st, const ProfHook& ph, double shift_rel = 0.0,
                             double* cert = nullptr);

struct FitParams {
  int n_iter, early_stop;
  double conv_tol, kappa, tie;
  int n_tol;
  double tol[16];
};
size_t fit_workspace_bytes(bool cplx, int batch, int D, int R);
NTU_HD int fit_stats_len(int n_iter, int D) { return 16 + 4 * n_iter + D; }
// guess (may be NULL: the fit computes it): the SVDU guess of every item
// from launch_svdu_guess with the same RX, RY, D and kappa
hipError_t launch_bond_fit(bool cplx, int batch, int D, int R, const void* g, const void* RX, const void* RY,
                           const FitParams& fp, void* MX, void* MY, double* stats, int stats_stride, void* ws,
                           hipStream_t st, const ProfHook& ph, const double* cert = nullptr,
                           const void* guess = nullptr);
// elements (compute type) of one item's SVDU guess
NTU_HD constexpr long long svdu_guess_elems() { return 2 * 20 * 20 + 1; }
hipError_t launch_svdu_guess(bool cplx, int batch, int D, int R, const void* RX, const void* RY, double kappa,
                             void* guess, hipStream_t st);

}  // namespace ntu
