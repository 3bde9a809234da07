// C ABI of libntu (declared in include/ntu.h): argument validation, the
// context's workspace, and the orchestration of a Trotter step.  Every
// numerical step runs in the HIP kernels of this library.
#include <stdio.h>
#include <string.h>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>
#include <algorithm>
#include <array>
#include "ntu.h"
#include "kernels.h"
#include "cell.h"
#include "mfma_gemm.h"

namespace {

struct Persist {
  // per-item persistent buffers of the Trotter step (compute type elements);
  // wA, wB: the compute-type copies of complex64 site tensors
  long long QX, QY, RX, RY, g, MX, MY, rA, rB, GA, GB, cert, guess, todo, wA, wB;
};

}  // namespace

struct ntu_ctx {
  int device = 0;
  int dtype = NTU_C128;
  bool cplx = true;
  int d = 2, na = 1, rg = 2, max_D = 1, max_batch = 1;
  hipStream_t stream = nullptr;
  // side stream of the Trotter step (default priority) and its fork / join
  // events; aux_user (when set) replaces the context's own aux
  hipStream_t aux = nullptr, aux_user = nullptr;
  hipEvent_t ev_fork = nullptr, ev_edges = nullptr, ev_red = nullptr, ev_join = nullptr;
  char* ws = nullptr;          // scratch of one call
  size_t ws_bytes = 0;
  char* step = nullptr;        // buffers of the Trotter step
  size_t step_bytes = 0;
  std::string err;
  // event profiler (ntu_profile_enable)
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_kind;
  int prof_n = 0;
  // tuned K split of the split-precision metric assembly per (D, precision)
  // (ntu_tune_env / ntu_set_env_ksplit); absent: the heuristic
  std::map<std::pair<int, int>, int> e6_ks;
  // tuned output tile width of the FP16X3 assembly per (D, precision)
  // (ntu_tune_env / ntu_set_env_tile); absent: the default
  std::map<std::pair<int, int>, int> e6_tile;
  // the Trotter step captured by ntu_trotter_step (opts.graph = 1) and the
  // arguments it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<char> graph_key;
};

// the context's stream, for the evolution run of api_ctm.hip
hipStream_t ntu_internal_ctx_stream(const ntu_ctx* c) { return c->stream; }

namespace {

thread_local std::string g_create_err;

// Stream captures of the caller that a context's Trotter step has joined
// (capture id -> context).  A step forks its side stream from the context
// stream and joins it back; one context inside a caller's capture is the
// supported case, a second context inside the same capture is refused.
std::mutex g_capture_mu;
std::map<unsigned long long, const ntu_ctx*> g_capture_owner;

bool claim_capture(const ntu_ctx* c, unsigned long long id) {
  std::lock_guard<std::mutex> lock(g_capture_mu);
  auto it = g_capture_owner.find(id);
  if (it != g_capture_owner.end()) return it->second == c;
  for (auto jt = g_capture_owner.begin(); jt != g_capture_owner.end();)
    jt = jt->second == c ? g_capture_owner.erase(jt) : std::next(jt);  // the context's earlier captures
  g_capture_owner[id] = c;
  return true;
}

void release_captures(const ntu_ctx* c) {
  std::lock_guard<std::mutex> lock(g_capture_mu);
  for (auto jt = g_capture_owner.begin(); jt != g_capture_owner.end();)
    jt = jt->second == c ? g_capture_owner.erase(jt) : std::next(jt);
}

ntu_status fail(ntu_ctx* c, ntu_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return s;
}

ntu_status hip_fail(ntu_ctx* c, hipError_t e, const char* where) {
  return fail(c, NTU_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

size_t elem_size(const ntu_ctx* c) { return c->cplx ? 16 : 8; }

// tuned K split of the metric assembly for (D, precision), 0 = heuristic
int env_ks_only(const ntu_ctx* c, int D, int precision) {
  auto it = c->e6_ks.find({D, precision});
  return it == c->e6_ks.end() ? 0 : it->second;
}
// tuned output tile width (columns) of the FP16X3 assembly, 0 = default
int env_tile(const ntu_ctx* c, int D, int precision) {
  auto it = c->e6_tile.find({D, precision});
  return it == c->e6_tile.end() ? 0 : it->second;
}
// the schedule handed to the environment contraction: K split in the low
// byte, tile width / 64 above it (0: the defaults)
int env_ks(const ntu_ctx* c, int D, int precision) {
  return env_ks_only(c, D, precision) | ((env_tile(c, D, precision) / 64) << 8);
}
int pdim(const ntu_ctx* c) { return c->d * c->na; }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

ntu_status check_common(ntu_ctx* c, int batch, int D) {
  if (!c) return NTU_ERR_ARG;
  c->err.clear();
  if (batch < 0) return fail(c, NTU_ERR_ARG, "batch must be >= 0");
  if (batch > c->max_batch) return fail(c, NTU_ERR_WORKSPACE, "batch exceeds the context's max_batch");
  if (D < 1 || D > c->max_D) return fail(c, NTU_ERR_SHAPE, "D outside [1, max_D] of the context");
  return NTU_OK;
}

size_t scratch_bytes(bool cplx, int batch, int p, int D, int rg) {
  const int R = D * rg;
  size_t a = 0;
  for (int prec = NTU_PREC_F64; prec <= NTU_PREC_BF16X6; ++prec)
    a = std::max(a, ntu::env_workspace_bytes(cplx, prec, batch, p, D, R));
  size_t b = ntu::fix_workspace_bytes(cplx, batch, R * R);
  size_t f = ntu::fit_workspace_bytes(cplx, batch, D, R);
  return std::max(a, std::max(b, f));
}

Persist persist_layout(int p, int D, int rg, int d) {
  const long long R = (long long)D * rg, D3 = (long long)D * D * D;
  Persist s;
  long long o = 0;
  s.QX = o; o += p * D3 * R;
  s.QY = o; o += p * D3 * R;
  s.RX = o; o += R * R;
  s.RY = o; o += R * R;
  s.g = o; o += R * R * R * R;
  s.MX = o; o += R * D;
  s.MY = o; o += R * D;
  s.rA = o; o += p * D3 * D;
  s.rB = o; o += p * D3 * D;
  s.GA = o; o += (long long)d * d * rg;
  s.GB = o; o += (long long)d * d * rg;
  s.cert = o; o += 1;  // the metric repair's certificate for the fit (one double per item)
  s.guess = o; o += ntu::svdu_guess_elems();  // the fit's SVDU guess, computed beside the environment
  s.todo = o; o += 1;  // the reduction's path flags, two ints per item
  s.wA = o; o += p * D3 * D;
  s.wB = o; o += p * D3 * D;
  (void)o;
  return s;
}
long long persist_elems(int p, int D, int rg, int d) {
  const long long R = (long long)D * rg, D3 = (long long)D * D * D;
  return 2 * p * D3 * R + 2 * R * R + R * R * R * R + 2 * R * D + 2 * p * D3 * D + 2LL * d * d * rg + 1 +
         ntu::svdu_guess_elems() + 1 + 2 * p * D3 * D;
}

const int PROF_CAP = 1 << 15;

void prof_mark(void* vc, int kind, int phase) {
  ntu_ctx* c = (ntu_ctx*)vc;
  if (!c->prof_on || c->prof_n >= PROF_CAP) return;
  if (hipEventRecord(c->prof_ev[c->prof_n], c->stream) != hipSuccess) return;
  c->prof_kind[c->prof_n] = kind * 2 + phase;
  ++c->prof_n;
}

ntu::ProfHook hook(ntu_ctx* c) {
  ntu::ProfHook h;
  h.mark = c->prof_on ? prof_mark : nullptr;
  h.ctx = c;
  return h;
}

const char* const PROF_NAMES[ntu::PK_COUNT] = {
    "rotate", "gate_split", "reduce_qr", "env_edges", "env_qprep", "env_left_right", "env_e4", "env_e5",
    "env_e6", "env_e6_reduce", "metric_herm", "metric_clip", "bond_fit", "recombine", "fit_certify"};

ntu::FitParams fit_params(const ntu_fit_opts* o) {
  ntu::FitParams fp{};
  fp.n_iter = o->n_iter;
  fp.early_stop = o->early_stop;
  fp.conv_tol = o->conv_tol;
  fp.kappa = o->kappa;
  fp.tie = o->tie;
  fp.n_tol = o->n_tol;
  for (int i = 0; i < 16; ++i) fp.tol[i] = o->tol[i];
  return fp;
}

ntu_status check_fit_opts(ntu_ctx* c, const ntu_fit_opts* o) {
  if (!o) return fail(c, NTU_ERR_ARG, "fit options are NULL");
  if (o->n_iter < 0 || o->n_iter > 1000) return fail(c, NTU_ERR_ARG, "n_iter outside [0, 1000]");
  if (o->n_tol < 1 || o->n_tol > 16) return fail(c, NTU_ERR_ARG, "n_tol outside [1, 16]");
  for (int i = 1; i < o->n_tol; ++i)
    if (!(o->tol[i] > o->tol[i - 1])) return fail(c, NTU_ERR_ARG, "tolerance ladder must ascend");
  if (!(o->tol[0] > 0)) return fail(c, NTU_ERR_ARG, "tolerances must be positive");
  if (!(o->kappa >= 0 && o->kappa < 1)) return fail(c, NTU_ERR_ARG, "kappa outside [0, 1)");
  return NTU_OK;
}


// ---------------------------------------------------------------------------
// descriptor checks
// ---------------------------------------------------------------------------
constexpr unsigned M_F64 = 1u << NTU_F64, M_C128 = 1u << NTU_C128, M_C64 = 1u << NTU_C64;

const char* dtype_name(int d) {
  return d == NTU_F64 ? "F64" : d == NTU_C128 ? "C128" : d == NTU_C64 ? "C64" : "unknown";
}

std::string shape_str(const long long* s, int n) {
  std::string o = "(";
  for (int i = 0; i < n; ++i) o += (i ? ", " : "") + std::to_string(s[i]);
  return o + ")";
}

unsigned compute_mask(const ntu_ctx* c) { return c->cplx ? M_C128 : M_F64; }

// t must be a dense row-major device array of the given shape and one of
// the element types in `dtypes`
ntu_status check_tensor(ntu_ctx* c, const ntu_tensor* t, const char* name, unsigned dtypes,
                        std::initializer_list<long long> want) {
  const std::string nm(name);
  if (!t) return fail(c, NTU_ERR_ARG, nm + ": NULL descriptor");
  if (!t->data) return fail(c, NTU_ERR_ARG, nm + ": NULL data pointer");
  if (t->dtype < 0 || t->dtype > NTU_C64 || !((dtypes >> t->dtype) & 1u)) {
    std::string ok;
    for (int d = 0; d <= NTU_C64; ++d)
      if ((dtypes >> d) & 1u) ok += std::string(ok.empty() ? "" : " or ") + dtype_name(d);
    return fail(c, NTU_ERR_DTYPE, nm + ": element type " + dtype_name(t->dtype) + ", expected " + ok);
  }
  const long long* w = want.begin();
  const int n = (int)want.size();
  if (t->ndim != n) {
    const int nd = t->ndim < 0 ? 0 : std::min(t->ndim, NTU_MAX_DIMS);
    long long got[NTU_MAX_DIMS];
    for (int i = 0; i < nd; ++i) got[i] = t->shape[i];
    return fail(c, NTU_ERR_SHAPE, nm + ": shape " + shape_str(got, nd) + ", expected " + shape_str(w, n));
  }
  for (int i = 0; i < n; ++i)
    if (t->shape[i] != w[i]) {
      long long got[NTU_MAX_DIMS];
      for (int k = 0; k < n; ++k) got[k] = t->shape[k];
      return fail(c, NTU_ERR_SHAPE, nm + ": shape " + shape_str(got, n) + ", expected " + shape_str(w, n));
    }
  long long st = 1;
  for (int i = n - 1; i >= 0; --i) {
    if (t->shape[i] != 1 && t->stride[i] != st)
      return fail(c, NTU_ERR_SHAPE, nm + ": not a dense row-major array (stride of dimension " + std::to_string(i) +
                                        " is " + std::to_string(t->stride[i]) + ", expected " + std::to_string(st) + ")");
    st *= t->shape[i];
  }
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, t->data) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, NTU_ERR_ARG, nm + ": not device memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(c, NTU_ERR_ARG, nm + ": not device memory");
  if (attr.device != c->device)
    return fail(c, NTU_ERR_ARG, nm + ": memory of device " + std::to_string(attr.device) + ", the context's is " +
                                    std::to_string(c->device));
  return NTU_OK;
}

// the bond dimension a descriptor implies at dimension `dim` (0 if absent)
int dim_of(const ntu_tensor* t, int dim) {
  if (!t || t->ndim <= dim || t->shape[dim] < 1 || t->shape[dim] > 64) return 0;
  return (int)t->shape[dim];
}

// the step graph captured by ntu_trotter_step, if any
void drop_graph(ntu_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_key.clear();
}

#define NTU_CHECK(x) do { ntu_status s_ = (x); if (s_) return s_; } while (0)

}  // namespace

namespace ntu {
void set_global_error(const char* msg) { g_create_err = msg; }
}  // namespace ntu

extern "C" {

const char* ntu_version(void) { return "libntu 0.1 (gfx950)"; }

void ntu_fit_opts_default(ntu_fit_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->n_iter = 20;
  o->early_stop = 0;
  o->conv_tol = 1e-12;
  o->kappa = 1e-10;
  o->n_tol = 8;
  for (int i = 0; i < 8; ++i) o->tol[i] = 1e-15 * pow(10.0, i);
  o->tie = 1e-15;
}

void ntu_step_opts_default(ntu_step_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->n_bonds = 4;
  o->order[0] = NTU_BOND_H1;
  o->order[1] = NTU_BOND_H2;
  o->order[2] = NTU_BOND_V1;
  o->order[3] = NTU_BOND_V2;
  o->precision = NTU_PREC_F64;
  o->fix_mode = NTU_FIX_HERM_CLIP;
  ntu_fit_opts_default(&o->fit);
  o->scheme = NTU_SCHEME_NTU;
}

ntu_status ntu_ctx_create(ntu_ctx** out, int device, int dtype, int d, int d_anc, int r_g, int max_D,
                          int max_batch) {
  if (!out) return fail(nullptr, NTU_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (dtype != NTU_F64 && dtype != NTU_C128) return fail(nullptr, NTU_ERR_DTYPE, "compute dtype must be F64 or C128");
  if (d < 1 || d > 4 || d_anc < 1 || d_anc > 4) return fail(nullptr, NTU_ERR_SHAPE, "d, d_anc must be in [1, 4]");
  if (r_g < 1 || r_g > d * d) return fail(nullptr, NTU_ERR_SHAPE, "r_g must be in [1, d^2]");
  if (max_D < 1 || max_D * r_g > 20) return fail(nullptr, NTU_ERR_SHAPE, "max_D * r_g must be in [1, 20]");
  if (max_batch < 1) return fail(nullptr, NTU_ERR_ARG, "max_batch must be >= 1");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, NTU_ERR_HIP, "no such HIP device");
  ntu_ctx* c = new ntu_ctx();
  c->device = device;
  c->dtype = dtype;
  c->cplx = dtype == NTU_C128;
  c->d = d; c->na = d_anc; c->rg = r_g; c->max_D = max_D; c->max_batch = max_batch;
  DeviceGuard guard(device);
  const int p = d * d_anc;
  size_t sb = 0;
  for (int D = 1; D <= max_D; ++D) sb = std::max(sb, scratch_bytes(c->cplx, max_batch, p, D, r_g));
  // the reduction's per-item path flags (both sides) also live at the start of the workspace
  c->ws_bytes = std::max(sb, 2 * (size_t)max_batch * sizeof(int) + 256);
  c->step_bytes = (size_t)persist_elems(p, max_D, r_g, d) * elem_size(c) * max_batch + 256;
  hipError_t e = hipMalloc((void**)&c->ws, c->ws_bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&c->step, c->step_bytes);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
  for (hipEvent_t* ev : {&c->ev_fork, &c->ev_edges, &c->ev_red, &c->ev_join})
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (c->ws) (void)hipFree(c->ws);
    if (c->step) (void)hipFree(c->step);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    for (hipEvent_t ev : {c->ev_fork, c->ev_edges, c->ev_red, c->ev_join})
      if (ev) (void)hipEventDestroy(ev);
    delete c;
    return fail(nullptr, NTU_ERR_HIP, std::string("context set-up failed: ") + hipGetErrorString(e));
  }
  *out = c;
  return NTU_OK;
}

ntu_status ntu_ctx_destroy(ntu_ctx* c) {
  if (!c) return NTU_ERR_ARG;
  DeviceGuard guard(c->device);
  release_captures(c);
  drop_graph(c);
  if (c->ws) (void)hipFree(c->ws);
  if (c->step) (void)hipFree(c->step);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  for (hipEvent_t ev : {c->ev_fork, c->ev_edges, c->ev_red, c->ev_join})
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : c->prof_ev) (void)hipEventDestroy(ev);
  delete c;
  return NTU_OK;
}

ntu_status ntu_set_stream(ntu_ctx* c, void* stream) {
  if (!c) return NTU_ERR_ARG;
  c->stream = (hipStream_t)stream;
  return NTU_OK;
}

ntu_status ntu_set_aux_stream(ntu_ctx* c, void* stream) {
  if (!c) return NTU_ERR_ARG;
  c->aux_user = (hipStream_t)stream;
  return NTU_OK;
}

const char* ntu_last_error(const ntu_ctx* c) {
  if (!c) return g_create_err.c_str();
  return c->err.c_str();
}

size_t ntu_workspace_bytes(const ntu_ctx* c) { return c ? c->ws_bytes + c->step_bytes : 0; }

ntu_status ntu_gate_split(ntu_ctx* c, int batch, const ntu_tensor* gate, ntu_tensor* GA, ntu_tensor* GB,
                          ntu_tensor* sigma) {
  NTU_CHECK(check_common(c, batch, 1));
  if (batch == 0) return NTU_OK;
  const long long d = c->d, r = c->rg;
  NTU_CHECK(check_tensor(c, gate, "gate", compute_mask(c), {batch, d * d, d * d}));
  NTU_CHECK(check_tensor(c, GA, "GA", compute_mask(c), {batch, d, d, r}));
  NTU_CHECK(check_tensor(c, GB, "GB", compute_mask(c), {batch, d, d, r}));
  NTU_CHECK(check_tensor(c, sigma, "sigma", M_F64, {batch, d * d}));
  DeviceGuard guard(c->device);
  const ntu::ProfHook ph = hook(c);
  ph(ntu::PK_GATE, 0);
  hipError_t e = ntu::launch_gate_split(c->cplx, batch, c->d, c->rg, gate->data, GA->data, GB->data,
                                        (double*)sigma->data, c->stream);
  ph(ntu::PK_GATE, 1);
  return e == hipSuccess ? NTU_OK : hip_fail(c, e, "gate_split");
}

ntu_status ntu_superop_gate(ntu_ctx* c, int batch, const ntu_tensor* gate, ntu_tensor* S) {
  NTU_CHECK(check_common(c, batch, 1));
  if (c->d != 4 || c->na != 1) return fail(c, NTU_ERR_SHAPE, "superop_gate needs a context with d = 4, d_anc = 1");
  if (batch == 0) return NTU_OK;
  NTU_CHECK(check_tensor(c, gate, "gate", M_F64 | M_C128, {batch, 4, 4}));
  NTU_CHECK(check_tensor(c, S, "S", M_F64, {batch, 16, 16}));
  DeviceGuard guard(c->device);
  const ntu::ProfHook ph = hook(c);
  ph(ntu::PK_GATE, 0);
  hipError_t e = ntu::launch_superop(gate->dtype == NTU_C128, batch, gate->data, (double*)S->data, c->stream);
  ph(ntu::PK_GATE, 1);
  return e == hipSuccess ? NTU_OK : hip_fail(c, e, "superop_gate");
}

ntu_status ntu_reduce_qr(ntu_ctx* c, int batch, const ntu_tensor* site, const ntu_tensor* gf, int side,
                         ntu_tensor* Q, ntu_tensor* R) {
  NTU_CHECK(check_common(c, batch, 1));
  if (side != 0 && side != 1) return fail(c, NTU_ERR_ARG, "side must be 0 (X) or 1 (Y)");
  if (batch == 0) return NTU_OK;
  const int D = dim_of(site, 2);
  NTU_CHECK(check_common(c, batch, D));
  const long long p = pdim(c), Rd = (long long)D * c->rg, D3 = (long long)D * D * D;
  NTU_CHECK(check_tensor(c, site, "site", compute_mask(c) | (c->cplx ? M_C64 : 0u), {batch, p, D, D, D, D}));
  NTU_CHECK(check_tensor(c, gf, "gate_factor", compute_mask(c), {batch, c->d, c->d, c->rg}));
  NTU_CHECK(check_tensor(c, Q, "Q", compute_mask(c), {batch, p * D3, Rd}));
  NTU_CHECK(check_tensor(c, R, "R", compute_mask(c), {batch, Rd, Rd}));
  DeviceGuard guard(c->device);
  const ntu::ProfHook ph = hook(c);
  ph(ntu::PK_REDUCE, 0);
  hipError_t e = ntu::launch_reduce_qr(c->cplx, site->dtype, batch, c->d, c->na, D, c->rg, site->data, gf->data,
                                       (long long)c->d * c->d * c->rg, side, Q->data, R->data, 1e-10, (int*)c->ws,
                                       c->stream);
  ph(ntu::PK_REDUCE, 1);
  return e == hipSuccess ? NTU_OK : hip_fail(c, e, "reduce_qr");
}

}  // extern "C"

namespace {
// operands of ntu_env_contract / ntu_tune_env; D from nbr[0]
ntu_status check_env_operands(ntu_ctx* c, int batch, const ntu_tensor* QX, const ntu_tensor* QY,
                              const ntu_tensor* nbr, const ntu_tensor* g, int* D_out) {
  if (!nbr) return fail(c, NTU_ERR_ARG, "nbr: NULL descriptor array");
  const int D = dim_of(&nbr[0], 2);
  NTU_CHECK(check_common(c, batch, D));
  const long long p = pdim(c), Rd = (long long)D * c->rg, D3 = (long long)D * D * D;
  NTU_CHECK(check_tensor(c, QX, "QX", compute_mask(c), {batch, p * D3, Rd}));
  NTU_CHECK(check_tensor(c, QY, "QY", compute_mask(c), {batch, p * D3, Rd}));
  static const char* const names[6] = {"nbr[0] (L)", "nbr[1] (TX)", "nbr[2] (BX)", "nbr[3] (TY)", "nbr[4] (BY)",
                                       "nbr[5] (Rn)"};
  for (int i = 0; i < 6; ++i) NTU_CHECK(check_tensor(c, &nbr[i], names[i], compute_mask(c), {batch, p, D, D, D, D}));
  NTU_CHECK(check_tensor(c, g, "g", compute_mask(c), {batch, Rd * Rd, Rd * Rd}));
  *D_out = D;
  return NTU_OK;
}
}  // namespace

extern "C" {

ntu_status ntu_env_contract(ntu_ctx* c, int batch, const ntu_tensor* QX, const ntu_tensor* QY,
                            const ntu_tensor nbr[6], int precision, ntu_tensor* g) {
  NTU_CHECK(check_common(c, batch, 1));
  if (precision < NTU_PREC_F64 || precision > NTU_PREC_BF16X6) return fail(c, NTU_ERR_ARG, "unknown precision");
  if (batch == 0) return NTU_OK;
  int D = 0;
  NTU_CHECK(check_env_operands(c, batch, QX, QY, nbr, g, &D));
  if (!ntu::env_precision_supported(c->cplx, precision, D))
    return fail(c, NTU_ERR_UNSUPPORTED, "precision not available for this dtype");
  const void* nb[6];
  for (int i = 0; i < 6; ++i) nb[i] = nbr[i].data;
  DeviceGuard guard(c->device);
  hipError_t e = ntu::launch_env_contract(c->cplx, precision, batch, pdim(c), D, D * c->rg, QX->data, QY->data, nb,
                                          g->data, c->ws, c->ws_bytes, c->stream, hook(c), 0,
                                          env_ks(c, D, precision));
  return e == hipSuccess ? NTU_OK : hip_fail(c, e, "env_contract");
}

ntu_status ntu_metric_fix(ntu_ctx* c, int batch, ntu_tensor* g, int mode, ntu_tensor* stats) {
  NTU_CHECK(check_common(c, batch, 1));
  if (mode != NTU_FIX_HERM && mode != NTU_FIX_HERM_CLIP) return fail(c, NTU_ERR_ARG, "unknown mode");
  if (batch == 0) return NTU_OK;
  if (!g || g->ndim != 3) return fail(c, NTU_ERR_SHAPE, "g: expected (batch, n, n)");
  // n = (D r_g)^2 for some D of the context
  int D = 0;
  for (int k = 1; k <= c->max_D; ++k)
    if ((long long)(k * c->rg) * (k * c->rg) == g->shape[1]) D = k;
  if (!D) return fail(c, NTU_ERR_SHAPE, "g: n is not (D r_g)^2 for a D of the context");
  const long long n = (long long)(D * c->rg) * (D * c->rg);
  NTU_CHECK(check_tensor(c, g, "g", compute_mask(c), {batch, n, n}));
  if (stats) NTU_CHECK(check_tensor(c, stats, "stats", M_F64, {batch, 8}));
  DeviceGuard guard(c->device);
  hipError_t e = ntu::launch_metric_fix(c->cplx, batch, (int)n, g->data, mode, stats ? (double*)stats->data : nullptr,
                                        8, c->ws, c->stream, hook(c));
  return e == hipSuccess ? NTU_OK : hip_fail(c, e, "metric_fix");
}

ntu_status ntu_bond_fit(ntu_ctx* c, int batch, const ntu_tensor* g, const ntu_tensor* RX, const ntu_tensor* RY,
                        const ntu_fit_opts* opts, ntu_tensor* MX, ntu_tensor* MY, ntu_tensor* stats) {
  NTU_CHECK(check_common(c, batch, 1));
  NTU_CHECK(check_fit_opts(c, opts));
  if (batch == 0) return NTU_OK;
  const int D = dim_of(MX, 2);
  NTU_CHECK(check_common(c, batch, D));
  const long long Rd = (long long)D * c->rg;
  NTU_CHECK(check_tensor(c, g, "g", compute_mask(c), {batch, Rd * Rd, Rd * Rd}));
  NTU_CHECK(check_tensor(c, RX, "RX", compute_mask(c), {batch, Rd, Rd}));
  NTU_CHECK(check_tensor(c, RY, "RY", compute_mask(c), {batch, Rd, Rd}));
  NTU_CHECK(check_tensor(c, MX, "MX", compute_mask(c), {batch, Rd, D}));
  NTU_CHECK(check_tensor(c, MY, "MY", compute_mask(c), {batch, Rd, D}));
  const int fl = ntu::fit_stats_len(opts->n_iter, D);
  if (stats) NTU_CHECK(check_tensor(c, stats, "stats", M_F64, {batch, fl}));
  DeviceGuard guard(c->device);
  hipError_t e = ntu::launch_bond_fit(c->cplx, batch, D, (int)Rd, g->data, RX->data, RY->data, fit_params(opts),
                                      MX->data, MY->data, stats ? (double*)stats->data : nullptr, fl, c->ws,
                                      c->stream, hook(c));
  return e == hipSuccess ? NTU_OK : hip_fail(c, e, "bond_fit");
}

ntu_status ntu_recombine(ntu_ctx* c, int batch, const ntu_tensor* QX, const ntu_tensor* QY, const ntu_tensor* MX,
                         const ntu_tensor* MY, ntu_tensor* Xn, ntu_tensor* Yn) {
  NTU_CHECK(check_common(c, batch, 1));
  if (batch == 0) return NTU_OK;
  const int D = dim_of(MX, 2);
  NTU_CHECK(check_common(c, batch, D));
  const long long p = pdim(c), Rd = (long long)D * c->rg, D3 = (long long)D * D * D;
  NTU_CHECK(check_tensor(c, QX, "QX", compute_mask(c), {batch, p * D3, Rd}));
  NTU_CHECK(check_tensor(c, QY, "QY", compute_mask(c), {batch, p * D3, Rd}));
  NTU_CHECK(check_tensor(c, MX, "MX", compute_mask(c), {batch, Rd, D}));
  NTU_CHECK(check_tensor(c, MY, "MY", compute_mask(c), {batch, Rd, D}));
  NTU_CHECK(check_tensor(c, Xn, "Xn", compute_mask(c), {batch, p, D, D, D, D}));
  NTU_CHECK(check_tensor(c, Yn, "Yn", compute_mask(c), {batch, p, D, D, D, D}));
  DeviceGuard guard(c->device);
  const ntu::ProfHook ph = hook(c);
  ph(ntu::PK_RECOMB, 0);
  hipError_t e = ntu::launch_recombine(c->cplx, batch, pdim(c), D, (int)Rd, QX->data, QY->data, MX->data, MY->data,
                                       Xn->data, Yn->data, 0, c->stream);
  ph(ntu::PK_RECOMB, 1);
  return e == hipSuccess ? NTU_OK : hip_fail(c, e, "recombine");
}

}  // extern "C"

namespace {

// The launches of one bond update over a batch of independent items: X, Y
// and the six neighbours nbr = [L, TX, BX, TY, BY, Rn] in the bond's
// canonical frame (compute type, item stride p D^4), the gate factors of item
// i at gA + i gf_item, gB + i gf_item; the new X, Y written to outX, outY
// (rotated back a quarter turn when vertical).  sb: the item-0 stats of this
// update (NTU_STEP_STATS_LEN doubles) with item stride s_item, or NULL.
hipError_t bond_launches(ntu_ctx* c, int batch, int D, const char* X, const char* Y, const void* const nbr[6],
                         const char* gA, const char* gB, long long gf_item, void* outX, void* outY, bool vertical,
                         const ntu_step_opts* opts, double* sb, long long s_item, const ntu::ProfHook& ph,
                         const char** where) {
  const bool cp = c->cplx;
  const int p = pdim(c), R = D * c->rg;
  const size_t el = elem_size(c);
  const Persist L = persist_layout(p, D, c->rg, c->d);
  auto buf = [&](long long off) -> char* { return c->step + (size_t)off * el * batch; };
  char* QX = buf(L.QX);
  char* QY = buf(L.QY);
  char* RX = buf(L.RX);
  char* RY = buf(L.RY);
  char* G = buf(L.g);
  char* MX = buf(L.MX);
  char* MY = buf(L.MY);
  double* cert = (double*)buf(L.cert);
  char* guess = buf(L.guess);
  int* todo = (int*)buf(L.todo);
  const ntu::FitParams fp = fit_params(&opts->fit);
  hipError_t e = hipSuccess;
  // Fork/join bookkeeping: once the side stream has been forked, every exit
  // joins it back into the context stream (an unjoined fork would leave the
  // side stream's work unordered with later calls, and would make a capture
  // that contains it invalid).
  bool forked = false;
  hipStream_t aux = c->aux_user ? c->aux_user : c->aux;
  auto join = [&]() {
    if (!forked) return;
    forked = false;
    if (hipEventRecord(c->ev_join, aux) == hipSuccess) (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
  };
#define NTU_STEP(x, what) do { e = (x); if (e != hipSuccess) { *where = what; join(); return e; } } while (0)
  if (opts->scheme == NTU_SCHEME_SVDU) {
    // SVDU update (Fig. 2): reduction, truncated SVD of RX RY^T, the fit's
    // balancing without a metric, recombination; all on the context stream
    ph(ntu::PK_REDUCE, 0);
    NTU_STEP(ntu::launch_reduce_qr_pair(cp, c->dtype, batch, c->d, c->na, D, c->rg, X, gA, Y, gB, gf_item, QX, RX, QY,
                                        RY, opts->fit.kappa, todo, c->stream), "reduce_qr");
    ph(ntu::PK_REDUCE, 1);
    NTU_STEP(ntu::launch_svdu_guess(cp, batch, D, R, RX, RY, opts->fit.kappa, guess, c->stream), "svdu_guess");
    NTU_STEP(ntu::launch_bond_fit(cp, batch, D, R, nullptr, RX, RY, fp, MX, MY, sb ? sb + 8 : nullptr, (int)s_item,
                                  c->ws, c->stream, ph, nullptr, guess), "bond_fit");
    ph(ntu::PK_RECOMB, 0);
    NTU_STEP(ntu::launch_recombine(cp, batch, p, D, R, QX, QY, MX, MY, outX, outY, vertical ? 1 : 0, c->stream),
             "recombine");
    ph(ntu::PK_RECOMB, 1);
    return hipSuccess;
  }
  // The side stream (aux) takes the work that does not need the reduction:
  // the edge tensors and transfers (they read only the neighbours) while
  // the reduction runs, then the fit's SVDU guess (it needs only RX, RY)
  // while the environment is contracted.  Events order the two streams.
  const ntu::ProfHook none{nullptr, nullptr};
  NTU_STEP(hipEventRecord(c->ev_fork, c->stream), "fork");
  NTU_STEP(hipStreamWaitEvent(aux, c->ev_fork, 0), "fork");
  forked = true;
  NTU_STEP(ntu::launch_env_contract(cp, opts->precision, batch, p, D, R, nullptr, nullptr, nbr, nullptr, c->ws,
                                    c->ws_bytes, aux, none, 1), "env_contract (edges)");
  NTU_STEP(hipEventRecord(c->ev_edges, aux), "fork");
  ph(ntu::PK_REDUCE, 0);
  NTU_STEP(ntu::launch_reduce_qr_pair(cp, c->dtype, batch, c->d, c->na, D, c->rg, X, gA, Y, gB, gf_item, QX, RX, QY,
                                      RY, opts->fit.kappa, todo, c->stream), "reduce_qr");
  ph(ntu::PK_REDUCE, 1);
  NTU_STEP(hipEventRecord(c->ev_red, c->stream), "fork");
  NTU_STEP(hipStreamWaitEvent(aux, c->ev_red, 0), "fork");
  NTU_STEP(ntu::launch_svdu_guess(cp, batch, D, R, RX, RY, opts->fit.kappa, guess, aux), "svdu_guess");
  NTU_STEP(hipStreamWaitEvent(c->stream, c->ev_edges, 0), "join");
  NTU_STEP(ntu::launch_env_contract(cp, opts->precision, batch, p, D, R, QX, QY, nbr, G, c->ws, c->ws_bytes,
                                    c->stream, ph, 2, env_ks(c, D, opts->precision)), "env_contract");
  // with the clip, the repair also tests the fit's certificate (g minus
  // 10 tau_max ||g||_F I positive definite, see the fit) and hands it over
  const bool clip = opts->fix_mode == NTU_FIX_HERM_CLIP;
  const double shift = 10.0 * fp.tol[fp.n_tol - 1];
  NTU_STEP(ntu::launch_metric_fix(cp, batch, R * R, G, opts->fix_mode, sb, (int)s_item, c->ws, c->stream, ph,
                                  clip ? shift : 0.0, clip ? cert : nullptr),
           "metric_fix");
  // the SVDU guess is ready: join the side stream
  NTU_STEP(hipEventRecord(c->ev_join, aux), "join");
  NTU_STEP(hipStreamWaitEvent(c->stream, c->ev_join, 0), "join");
  forked = false;
  NTU_STEP(ntu::launch_bond_fit(cp, batch, D, R, G, RX, RY, fp, MX, MY, sb ? sb + 8 : nullptr, (int)s_item, c->ws,
                                c->stream, ph, clip ? cert : nullptr, guess), "bond_fit");
  ph(ntu::PK_RECOMB, 0);
  NTU_STEP(ntu::launch_recombine(cp, batch, p, D, R, QX, QY, MX, MY, outX, outY, vertical ? 1 : 0, c->stream),
           "recombine");
  ph(ntu::PK_RECOMB, 1);
#undef NTU_STEP
  return hipSuccess;
}

// The launches of one Trotter step (everything after argument checks).  A, B
// are compute-type site tensors; for complex64 storage (c64) the caller's
// tensors are A64, B64 and A, B are the context's working copies.
hipError_t step_launches(ntu_ctx* c, int batch, int D, char* A, char* B, void* A64, void* B64, bool c64,
                         const char* gate_factors, const ntu_step_opts* opts, double* stats, const ntu::ProfHook& ph,
                         const char** where) {
  const bool cp = c->cplx;
  const int p = pdim(c);
  const size_t el = elem_size(c);
  const Persist L = persist_layout(p, D, c->rg, c->d);
  auto buf = [&](long long off) -> char* { return c->step + (size_t)off * el * batch; };
  char* rA = buf(L.rA);
  char* rB = buf(L.rB);
  const long long gfs = (long long)c->d * c->d * c->rg;  // elements of one factor
  const long long gf_item = 8 * gfs;                      // 4 bonds x (GA, GB)
  const int sl = 8 + ntu::fit_stats_len(opts->fit.n_iter, D);
  const long long s_item = (long long)opts->n_bonds * sl;
  const long long nsite = (long long)p * D * D * D * D;
  hipError_t e = hipSuccess;
#define NTU_STEP(x, what) do { e = (x); if (e != hipSuccess) { *where = what; return e; } } while (0)
  if (c64) {
    NTU_STEP(ntu::launch_cast_c64(batch * nsite, A64, A, 0, c->stream), "complex64 load");
    NTU_STEP(ntu::launch_cast_c64(batch * nsite, B64, B, 0, c->stream), "complex64 load");
  }
  for (int bi = 0; bi < opts->n_bonds; ++bi) {
    const int bond = opts->order[bi];
    const bool vertical = bond >= 2, x_is_a = (bond == NTU_BOND_H1 || bond == NTU_BOND_V1);
    char* a = A;
    char* b = B;
    if (vertical) {
      ph(ntu::PK_ROTATE, 0);
      NTU_STEP(ntu::launch_rotate_cw(cp, batch, p, D, A, rA, c->stream), "rotate");
      NTU_STEP(ntu::launch_rotate_cw(cp, batch, p, D, B, rB, c->stream), "rotate");
      ph(ntu::PK_ROTATE, 1);
      a = rA;
      b = rB;
    }
    char* X = x_is_a ? a : b;
    char* Y = x_is_a ? b : a;
    const char* gA = gate_factors + (size_t)(bond * 2 + 0) * gfs * el;
    const char* gB = gate_factors + (size_t)(bond * 2 + 1) * gfs * el;
    // new X -> (A or B), new Y -> the other, rotated back for vertical bonds
    void* outX = x_is_a ? A : B;
    void* outY = x_is_a ? B : A;
    double* sb = stats ? stats + (size_t)bi * sl : nullptr;
    // on the two-site checkerboard X's neighbours are of Y's type and vice versa
    const void* nbr[6] = {Y, Y, Y, X, X, X};
    NTU_STEP(bond_launches(c, batch, D, X, Y, nbr, gA, gB, gf_item, outX, outY, vertical, opts, sb, s_item, ph, where),
             *where);
  }
  if (c64) {
    NTU_STEP(ntu::launch_cast_c64(batch * nsite, A, A64, 1, c->stream), "complex64 store");
    NTU_STEP(ntu::launch_cast_c64(batch * nsite, B, B64, 1, c->stream), "complex64 store");
  }
#undef NTU_STEP
  return hipSuccess;
}

// the arguments a captured step depends on, as bytes (fields copied one by
// one, so padding never enters the comparison)
std::vector<char> step_key(int batch, int D, const void* A, const void* B, int a_dtype, const void* gf,
                           const void* stats, const ntu_step_opts* o) {
  std::vector<char> k;
  auto put = [&](const void* p, size_t n) { k.insert(k.end(), (const char*)p, (const char*)p + n); };
  put(&batch, sizeof batch); put(&D, sizeof D); put(&A, sizeof A); put(&B, sizeof B); put(&a_dtype, sizeof a_dtype);
  put(&gf, sizeof gf); put(&stats, sizeof stats);
  put(&o->n_bonds, sizeof(int)); put(o->order, sizeof o->order); put(&o->precision, sizeof(int));
  put(&o->fix_mode, sizeof(int)); put(&o->scheme, sizeof(int));
  const ntu_fit_opts& f = o->fit;
  put(&f.n_iter, sizeof(int)); put(&f.early_stop, sizeof(int)); put(&f.conv_tol, sizeof(double));
  put(&f.kappa, sizeof(double)); put(&f.n_tol, sizeof(int)); put(f.tol, sizeof f.tol); put(&f.tie, sizeof(double));
  return k;
}

}  // namespace

extern "C" {

ntu_status ntu_trotter_step(ntu_ctx* c, int batch, ntu_tensor* A, ntu_tensor* B, const ntu_tensor* gate_factors,
                            const ntu_step_opts* opts, ntu_tensor* stats) {
  NTU_CHECK(check_common(c, batch, 1));
  if (!opts) return fail(c, NTU_ERR_ARG, "step options are NULL");
  if (opts->n_bonds < 0 || opts->n_bonds > 8) return fail(c, NTU_ERR_ARG, "n_bonds outside [0, 8]");
  for (int i = 0; i < opts->n_bonds; ++i)
    if (opts->order[i] < 0 || opts->order[i] > 3) return fail(c, NTU_ERR_ARG, "unknown bond in order");
  if (opts->precision < NTU_PREC_F64 || opts->precision > NTU_PREC_BF16X6) return fail(c, NTU_ERR_ARG, "unknown precision");
  if (opts->fix_mode != NTU_FIX_HERM && opts->fix_mode != NTU_FIX_HERM_CLIP) return fail(c, NTU_ERR_ARG, "unknown fix mode");
  NTU_CHECK(check_fit_opts(c, &opts->fit));
  if (opts->scheme != NTU_SCHEME_NTU && opts->scheme != NTU_SCHEME_SVDU) return fail(c, NTU_ERR_ARG, "unknown scheme");
  if (opts->graph != 0 && opts->graph != 1) return fail(c, NTU_ERR_ARG, "graph must be 0 or 1");
  if (batch == 0 || opts->n_bonds == 0) return NTU_OK;
  const int D = dim_of(A, 2);
  NTU_CHECK(check_common(c, batch, D));
  const long long p = pdim(c);
  const unsigned site_types = compute_mask(c) | (c->cplx ? M_C64 : 0u);
  NTU_CHECK(check_tensor(c, A, "A", site_types, {batch, p, D, D, D, D}));
  NTU_CHECK(check_tensor(c, B, "B", 1u << A->dtype, {batch, p, D, D, D, D}));
  NTU_CHECK(check_tensor(c, gate_factors, "gate_factors", compute_mask(c), {batch, 4, 2, c->d, c->d, c->rg}));
  const int fl = ntu::fit_stats_len(opts->fit.n_iter, D);
  if (stats) NTU_CHECK(check_tensor(c, stats, "stats", M_F64, {batch, opts->n_bonds, 8 + fl}));
  if (opts->scheme == NTU_SCHEME_NTU && !ntu::env_precision_supported(c->cplx, opts->precision, D))
    return fail(c, NTU_ERR_UNSUPPORTED, "precision not available for this dtype");
  if (A->data == B->data) return fail(c, NTU_ERR_ARG, "A and B alias");
  DeviceGuard guard(c->device);
  const bool c64 = A->dtype == NTU_C64;
  const Persist L = persist_layout((int)p, D, c->rg, c->d);
  const size_t el = elem_size(c);
  char* wa = c64 ? c->step + (size_t)L.wA * el * batch : (char*)A->data;
  char* wb = c64 ? c->step + (size_t)L.wB * el * batch : (char*)B->data;
  double* st = stats ? (double*)stats->data : nullptr;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  unsigned long long cap_id = 0;
  hipError_t e = hipStreamGetCaptureInfo(c->stream, &cs, &cap_id);
  if (e != hipSuccess) return hip_fail(c, e, "stream capture query");
  const bool capturing = cs != hipStreamCaptureStatusNone;
  if (capturing && cs != hipStreamCaptureStatusActive) return fail(c, NTU_ERR_ARG, "the caller's capture is invalidated");
  // one context per caller capture: a second context's fork and join inside
  // the same capture is not a supported configuration
  if (capturing && !opts->graph && !claim_capture(c, cap_id))
    return fail(c, NTU_ERR_UNSUPPORTED, "another context's Trotter step is already part of this stream capture");
  const char* where = "";
  if (!opts->graph) {
    // eager (possibly inside the caller's own capture: no profiler events then)
    e = step_launches(c, batch, D, wa, wb, A->data, B->data, c64, (const char*)gate_factors->data, opts, st,
                      capturing ? ntu::ProfHook{nullptr, nullptr} : hook(c), &where);
    return e == hipSuccess ? NTU_OK : hip_fail(c, e, where);
  }
  if (capturing) return fail(c, NTU_ERR_ARG, "graph = 1 while the context stream is being captured by the caller");
  if (!c->stream) return fail(c, NTU_ERR_ARG, "graph = 1 needs a context stream other than the null stream");
  std::vector<char> key = step_key(batch, D, A->data, B->data, A->dtype, gate_factors->data, st, opts);
  if (!c->graph_exec || key != c->graph_key) {
    drop_graph(c);
    e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(c, e, "begin capture");
    hipError_t el_ = step_launches(c, batch, D, wa, wb, A->data, B->data, c64, (const char*)gate_factors->data, opts,
                                   st, ntu::ProfHook{nullptr, nullptr}, &where);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->stream, &g);
    if (el_ != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      return el_ != hipSuccess ? hip_fail(c, el_, where) : hip_fail(c, e, "end capture");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(c, e, "graph instantiate");
    }
    c->graph = g;
    c->graph_exec = x;
    c->graph_key.swap(key);
  }
  e = hipGraphLaunch(c->graph_exec, c->stream);
  return e == hipSuccess ? NTU_OK : hip_fail(c, e, "graph launch");
}

ntu_status ntu_cell_step(ntu_ctx* c, int Lx, int Ly, ntu_tensor* T, int n_bonds, const int* bonds,
                         const ntu_tensor* gate_factors, const ntu_step_opts* opts, ntu_tensor* work,
                         ntu_tensor* stats, int* n_groups) {
  NTU_CHECK(check_common(c, 1, 1));
  if (n_groups) *n_groups = 0;
  if (!opts) return fail(c, NTU_ERR_ARG, "step options are NULL");
  if (opts->precision < NTU_PREC_F64 || opts->precision > NTU_PREC_BF16X6) return fail(c, NTU_ERR_ARG, "unknown precision");
  if (opts->fix_mode != NTU_FIX_HERM && opts->fix_mode != NTU_FIX_HERM_CLIP) return fail(c, NTU_ERR_ARG, "unknown fix mode");
  NTU_CHECK(check_fit_opts(c, &opts->fit));
  if (opts->scheme != NTU_SCHEME_NTU && opts->scheme != NTU_SCHEME_SVDU) return fail(c, NTU_ERR_ARG, "unknown scheme");
  if (Lx < 2 || Ly < 2 || (long long)Lx * Ly > 4096) return fail(c, NTU_ERR_SHAPE, "cell: Lx, Ly >= 2 and Lx Ly <= 4096");
  if (n_bonds < 0 || n_bonds > 65536) return fail(c, NTU_ERR_ARG, "n_bonds outside [0, 65536]");
  if (n_bonds > 0 && !bonds) return fail(c, NTU_ERR_ARG, "bonds is NULL");
  for (int k = 0; k < n_bonds; ++k) {
    const int x = bonds[3 * k], y = bonds[3 * k + 1], dir = bonds[3 * k + 2];
    if (x < 0 || x >= Lx || y < 0 || y >= Ly || (dir != 0 && dir != 1))
      return fail(c, NTU_ERR_ARG, "bond " + std::to_string(k) + ": x in [0, Lx), y in [0, Ly), dir 0 or 1");
  }
  if (n_bonds == 0) return NTU_OK;
  const int D = dim_of(T, 2);
  NTU_CHECK(check_common(c, 1, D));
  const long long p = pdim(c);
  const long long nsite = p * D * D * D * D;
  NTU_CHECK(check_tensor(c, T, "T", compute_mask(c), {(long long)Lx * Ly, p, D, D, D, D}));
  NTU_CHECK(check_tensor(c, gate_factors, "gate_factors", compute_mask(c), {n_bonds, 2, c->d, c->d, c->rg}));
  const int G = std::min(c->max_batch, ntu::CELL_GROUP_MAX);
  if (!work || work->ndim != 1) return fail(c, NTU_ERR_SHAPE, "work: a one-dimensional array");
  NTU_CHECK(check_tensor(c, work, "work", compute_mask(c), {work->shape[0]}));
  if (work->shape[0] < 8 * G * nsite)
    return fail(c, NTU_ERR_WORKSPACE, "work: " + std::to_string(8 * G * nsite) + " elements needed (8 min(max_batch, " +
                                          std::to_string(ntu::CELL_GROUP_MAX) + ") p D^4)");
  const int sl = 8 + ntu::fit_stats_len(opts->fit.n_iter, D);
  if (stats) NTU_CHECK(check_tensor(c, stats, "stats", M_F64, {n_bonds, sl}));
  if (opts->scheme == NTU_SCHEME_NTU && !ntu::env_precision_supported(c->cplx, opts->precision, D))
    return fail(c, NTU_ERR_UNSUPPORTED, "precision not available for this dtype");
  DeviceGuard guard(c->device);
  // cluster sites [X, Y, L, TX, BX, TY, BY, Rn] of every bond, in the bond's
  // frame (vertical bonds: the lattice turned a quarter turn clockwise, so
  // left is below, up is left)
  auto site = [&](int i, int j) { return ((i % Lx) + Lx) % Lx + Lx * (((j % Ly) + Ly) % Ly); };
  std::vector<std::array<int, 8>> cl(n_bonds);
  for (int k = 0; k < n_bonds; ++k) {
    const int x = bonds[3 * k], y = bonds[3 * k + 1];
    if (bonds[3 * k + 2] == 0)
      cl[k] = {site(x, y), site(x + 1, y), site(x - 1, y), site(x, y + 1), site(x, y - 1), site(x + 1, y + 1),
               site(x + 1, y - 1), site(x + 2, y)};
    else
      cl[k] = {site(x, y), site(x, y + 1), site(x, y - 1), site(x - 1, y), site(x + 1, y), site(x - 1, y + 1),
               site(x + 1, y + 1), site(x, y + 2)};
  }
  // two updates commute when neither changes a site of the other's cluster
  auto independent = [&](int a, int b) {
    for (int u = 0; u < 2; ++u)
      for (int r = 0; r < 8; ++r)
        if (cl[a][u] == cl[b][r] || cl[b][u] == cl[a][r]) return false;
    return true;
  };
  const size_t el = elem_size(c);
  const long long gfs = (long long)c->d * c->d * c->rg;
  char* W = (char*)work->data;
  const char* GF = (const char*)gate_factors->data;
  double* st = stats ? (double*)stats->data : nullptr;
  const ntu::ProfHook ph = hook(c);
  int groups = 0;
  for (int k0 = 0; k0 < n_bonds;) {
    int k1 = k0 + 1;
    while (k1 < n_bonds && k1 - k0 < G) {
      bool ok = true;
      for (int j = k0; j < k1 && ok; ++j) ok = independent(j, k1);
      if (!ok) break;
      ++k1;
    }
    ntu::CellGroup g{};
    g.n = k1 - k0;
    for (int k = 0; k < g.n; ++k) {
      for (int r = 0; r < 8; ++r) g.site[k][r] = cl[k0 + k][r];
      g.vert[k] = bonds[3 * (k0 + k) + 2];
    }
    auto role = [&](int r) { return W + (size_t)r * g.n * nsite * el; };
    hipError_t e = ntu::launch_cell_gather(c->cplx, T->data, W, (int)p, D, g, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "cell gather");
    const void* nbr[6] = {role(2), role(3), role(4), role(5), role(6), role(7)};
    const char* where = "";
    // the new X, Y are written over roles 0 and 1 in the bond's frame (the
    // reduction has read them by then) and turned back by the scatter
    e = bond_launches(c, g.n, D, role(0), role(1), nbr, GF + (size_t)(2 * k0) * gfs * el,
                      GF + (size_t)(2 * k0 + 1) * gfs * el, 2 * gfs, role(0), role(1), false, opts,
                      st ? st + (size_t)k0 * sl : nullptr, sl, ph, &where);
    if (e != hipSuccess) return hip_fail(c, e, where);
    e = ntu::launch_cell_scatter(c->cplx, T->data, W, (int)p, D, g, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "cell scatter");
    ++groups;
    k0 = k1;
  }
  if (n_groups) *n_groups = groups;
  return NTU_OK;
}

ntu_status ntu_tune_env(ntu_ctx* c, int batch, int precision, const ntu_tensor* QX, const ntu_tensor* QY,
                        const ntu_tensor nbr[6], ntu_tensor* g, int reps, int* best_ks, float* best_ms) {
  NTU_CHECK(check_common(c, batch, 1));
  if (precision != NTU_PREC_BF16X3 && precision != NTU_PREC_BF16X6 && precision != NTU_PREC_FP16X3)
    return fail(c, NTU_ERR_ARG, "tuning applies to the split precisions");
  if (reps < 1) return fail(c, NTU_ERR_ARG, "reps < 1");
  if (batch == 0) return NTU_OK;
  int D = 0;
  NTU_CHECK(check_env_operands(c, batch, QX, QY, nbr, g, &D));
  if (!ntu::env_precision_supported(c->cplx, precision, D))
    return fail(c, NTU_ERR_UNSUPPORTED, "precision not available for this dtype");
  const void* nb[6];
  for (int i = 0; i < 6; ++i) nb[i] = nbr[i].data;
  DeviceGuard guard(c->device);
  const int R = D * c->rg;
  const int kdef = ntu::e6_ksplit_default(c->cplx, batch, R, D), kcap = ntu::e6_ksplit_max(c->cplx, batch, R, D);
  std::vector<int> ks_cand;
  for (int k = 1; k <= std::min(kcap, ntu::E6_KS_TUNE_MAX); ++k) ks_cand.push_back(k);
  if (kdef > ntu::E6_KS_TUNE_MAX) ks_cand.push_back(kdef);
  // candidates: (K split, tile width) as the schedule code of env_ks; the
  // tile width is a choice of the FP16X3 assembly only
  std::vector<int> tiles = {0};
  if (precision == NTU_PREC_FP16X3) tiles = {128, 256};
  std::vector<int> cand;
  for (int t : tiles)
    for (int k : ks_cand) cand.push_back(k | ((t / 64) << 8));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int best = kdef | ((tiles[0] / 64) << 8);
  float tbest = -1.0f;
  const ntu::ProfHook none{nullptr, nullptr};
  for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
    auto launch = [&]() {
      return ntu::launch_env_contract(c->cplx, precision, batch, pdim(c), D, R, QX->data, QY->data, nb, g->data,
                                      c->ws, c->ws_bytes, c->stream, none, 0, cand[i]);
    };
    e = launch();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    ms /= reps;
    if (e == hipSuccess && (tbest < 0.0f || ms < tbest)) {
      tbest = ms;
      best = cand[i];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(c, e, "tune_env");
  c->e6_ks[{D, precision}] = best & 0xff;
  if (best >> 8) c->e6_tile[{D, precision}] = (best >> 8) * 64;
  else c->e6_tile.erase({D, precision});
  if (best_ks) *best_ks = best & 0xff;
  if (best_ms) *best_ms = tbest;
  return NTU_OK;
}

ntu_status ntu_set_env_ksplit(ntu_ctx* c, int D, int precision, int ks) {
  if (!c) return NTU_ERR_ARG;
  if (D < 1 || D > c->max_D) return fail(c, NTU_ERR_SHAPE, "D outside [1, max_D]");
  if (precision != NTU_PREC_BF16X3 && precision != NTU_PREC_BF16X6 && precision != NTU_PREC_FP16X3)
    return fail(c, NTU_ERR_ARG, "the K split applies to the split precisions");
  if (ks < 0) return fail(c, NTU_ERR_ARG, "ks < 0");
  if (ks == 0) c->e6_ks.erase({D, precision});
  else c->e6_ks[{D, precision}] = ks;
  return NTU_OK;
}

int ntu_get_env_ksplit(ntu_ctx* c, int D, int precision) {
  if (!c) return NTU_ERR_ARG;
  return env_ks_only(c, D, precision);
}

ntu_status ntu_set_env_tile(ntu_ctx* c, int D, int precision, int width) {
  if (!c) return NTU_ERR_ARG;
  if (D < 1 || D > c->max_D) return fail(c, NTU_ERR_SHAPE, "D outside [1, max_D]");
  if (precision != NTU_PREC_FP16X3) return fail(c, NTU_ERR_ARG, "the tile width applies to NTU_PREC_FP16X3");
  if (width != 0 && width != 128 && width != 256) return fail(c, NTU_ERR_ARG, "tile width must be 0, 128 or 256");
  if (width == 0) c->e6_tile.erase({D, precision});
  else c->e6_tile[{D, precision}] = width;
  return NTU_OK;
}

int ntu_get_env_tile(ntu_ctx* c, int D, int precision) {
  if (!c) return NTU_ERR_ARG;
  return env_tile(c, D, precision);
}

ntu_status ntu_tune_save(ntu_ctx* c, const char* path) {
  if (!c || !path) return NTU_ERR_ARG;
  FILE* f = fopen(path, "w");
  if (!f) return fail(c, NTU_ERR_ARG, std::string("cannot write ") + path);
  fprintf(f, "# D precision e6_ksplit tile_width\n");
  std::map<std::pair<int, int>, std::pair<int, int>> rows;
  for (const auto& kv : c->e6_ks) rows[kv.first].first = kv.second;
  for (const auto& kv : c->e6_tile) rows[kv.first].second = kv.second;
  for (const auto& kv : rows)
    fprintf(f, "%d %d %d %d\n", kv.first.first, kv.first.second, kv.second.first, kv.second.second);
  const bool ok = fclose(f) == 0;
  return ok ? NTU_OK : fail(c, NTU_ERR_ARG, std::string("cannot write ") + path);
}

ntu_status ntu_tune_load(ntu_ctx* c, const char* path) {
  if (!c || !path) return NTU_ERR_ARG;
  FILE* f = fopen(path, "r");
  if (!f) return fail(c, NTU_ERR_ARG, std::string("cannot read ") + path);
  char line[256];
  ntu_status s = NTU_OK;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int D = 0, prec = 0, ks = 0, tile = 0;
    const int got = sscanf(line, "%d %d %d %d", &D, &prec, &ks, &tile);
    if (got < 3 || ks < 0 || (got == 4 && tile != 0 && tile != 128 && tile != 256)) {
      s = fail(c, NTU_ERR_ARG, std::string("malformed line in ") + path);
      break;
    }
    if (D >= 1 && D <= c->max_D && (prec == NTU_PREC_BF16X3 || prec == NTU_PREC_BF16X6 || prec == NTU_PREC_FP16X3)) {
      if (ks > 0) c->e6_ks[{D, prec}] = ks;
      if (got == 4 && tile > 0 && prec == NTU_PREC_FP16X3) c->e6_tile[{D, prec}] = tile;
    }
  }
  fclose(f);
  return s;
}

ntu_status ntu_profile_enable(ntu_ctx* c, int on) {
  if (!c) return NTU_ERR_ARG;
  DeviceGuard guard(c->device);
  if (on && c->prof_ev.empty()) {
    c->prof_ev.resize(PROF_CAP);
    c->prof_kind.resize(PROF_CAP);
    for (int i = 0; i < PROF_CAP; ++i) {
      hipError_t e = hipEventCreate(&c->prof_ev[i]);
      if (e != hipSuccess) return hip_fail(c, e, "profile events");
    }
  }
  c->prof_on = on != 0;
  c->prof_n = 0;
  return NTU_OK;
}

int ntu_profile_read(ntu_ctx* c, double* ms, int* count, int n) {
  if (!c || n < 0) return NTU_ERR_ARG;
  DeviceGuard guard(c->device);
  for (int k = 0; k < n; ++k) { if (ms) ms[k] = 0.0; if (count) count[k] = 0; }
  if (c->prof_n > 0) (void)hipEventSynchronize(c->prof_ev[c->prof_n - 1]);
  int open_idx[ntu::PK_COUNT];
  for (int k = 0; k < ntu::PK_COUNT; ++k) open_idx[k] = -1;
  for (int i = 0; i < c->prof_n; ++i) {
    int kind = c->prof_kind[i] / 2, phase = c->prof_kind[i] % 2;
    if (phase == 0) { open_idx[kind] = i; continue; }
    if (open_idx[kind] < 0) continue;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, c->prof_ev[open_idx[kind]], c->prof_ev[i]) == hipSuccess && kind < n) {
      if (ms) ms[kind] += t;
      if (count) count[kind] += 1;
    }
    open_idx[kind] = -1;
  }
  c->prof_n = 0;
  return ntu::PK_COUNT;
}

const char* ntu_profile_kind_name(int kind) {
  return (kind >= 0 && kind < ntu::PK_COUNT) ? PROF_NAMES[kind] : "";
}

}  // extern "C"
