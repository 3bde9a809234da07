"""Python binding of libntu (C ABI in ``include/ntu.h``).

Argument marshalling only: every numerical step runs in the HIP kernels of
``libntu.so``.  Tensors are torch tensors on the GPU; outputs are allocated
with torch (device memory) and filled by the library on the current torch
stream.  There is no fallback: if the library is missing, or the library
rejects a tensor (element type, shape, strides, memory that is not on the
context's GPU), the call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libntu.so")

NTU_OK = 0
F64, C128, C64 = 0, 1, 2
PREC_F64, PREC_BF16X3, PREC_FP16X3, PREC_BF16X6 = 0, 1, 2, 3
FIX_HERM, FIX_HERM_CLIP = 0, 1
BOND_H1, BOND_H2, BOND_V1, BOND_V2 = 0, 1, 2, 3
PRECISIONS = {"f64": PREC_F64, "bf16x3": PREC_BF16X3, "fp16x3": PREC_FP16X3, "bf16x6": PREC_BF16X6}
SCHEME_NTU, SCHEME_SVDU = 0, 1
SCHEMES = {"ntu": SCHEME_NTU, "svdu": SCHEME_SVDU}

EXPORTED = (
    "ntu_ctx_create", "ntu_ctx_destroy", "ntu_set_stream", "ntu_set_aux_stream", "ntu_last_error",
    "ntu_workspace_bytes",
    "ntu_version", "ntu_gate_split", "ntu_reduce_qr", "ntu_env_contract", "ntu_metric_fix",
    "ntu_fit_opts_default", "ntu_bond_fit", "ntu_recombine", "ntu_step_opts_default", "ntu_trotter_step",
    "ntu_profile_enable", "ntu_profile_read", "ntu_profile_kind_name",
    "ntu_tune_env", "ntu_set_env_ksplit", "ntu_get_env_ksplit", "ntu_set_env_tile", "ntu_get_env_tile",
    "ntu_tune_save", "ntu_tune_load",
    "ntu_metric_fix_noalloc", "ntu_superop_gate",
    "ntu_ctm_create", "ntu_ctm_destroy", "ntu_ctm_set_stream", "ntu_ctm_last_error", "ntu_ctm_run", "ntu_ctm_expect",
    "ntu_evolve", "ntu_cell_step",
)


class FitOpts(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int), ("early_stop", ctypes.c_int), ("conv_tol", ctypes.c_double),
                ("kappa", ctypes.c_double), ("n_tol", ctypes.c_int), ("tol", ctypes.c_double * 16),
                ("tie", ctypes.c_double)]


class StepOpts(ctypes.Structure):
    _fields_ = [("n_bonds", ctypes.c_int), ("order", ctypes.c_int * 8), ("precision", ctypes.c_int),
                ("fix_mode", ctypes.c_int), ("fit", FitOpts), ("scheme", ctypes.c_int), ("graph", ctypes.c_int)]


class EvolveOpts(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int), ("measure_every", ctypes.c_int), ("ctm_iters", ctypes.c_int),
                ("ctm_continue", ctypes.c_int), ("energy_tol", ctypes.c_double)]


MAX_DIMS = 8


class Tensor(ctypes.Structure):
    """``ntu_tensor``: data pointer, element type, shape and strides (elements)."""
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("ndim", ctypes.c_int32),
                ("shape", ctypes.c_int64 * MAX_DIMS), ("stride", ctypes.c_int64 * MAX_DIMS)]


_lib = None


def load():
    """Load libntu.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    L.ntu_ctx_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, i32, i32, i32]
    L.ntu_ctx_destroy.argtypes = [vp]
    L.ntu_set_stream.argtypes = [vp, vp]
    L.ntu_set_aux_stream.argtypes = [vp, vp]
    L.ntu_last_error.argtypes = [vp]
    L.ntu_last_error.restype = ctypes.c_char_p
    L.ntu_workspace_bytes.argtypes = [vp]
    L.ntu_workspace_bytes.restype = ctypes.c_size_t
    L.ntu_version.restype = ctypes.c_char_p
    tp = ctypes.POINTER(Tensor)
    L.ntu_gate_split.argtypes = [vp, i32, tp, tp, tp, tp]
    L.ntu_reduce_qr.argtypes = [vp, i32, tp, tp, i32, tp, tp]
    L.ntu_env_contract.argtypes = [vp, i32, tp, tp, tp, i32, tp]
    L.ntu_metric_fix.argtypes = [vp, i32, tp, i32, tp]
    L.ntu_fit_opts_default.argtypes = [ctypes.POINTER(FitOpts)]
    L.ntu_fit_opts_default.restype = None
    L.ntu_bond_fit.argtypes = [vp, i32, tp, tp, tp, ctypes.POINTER(FitOpts), tp, tp, tp]
    L.ntu_recombine.argtypes = [vp, i32, tp, tp, tp, tp, tp, tp]
    L.ntu_step_opts_default.argtypes = [ctypes.POINTER(StepOpts)]
    L.ntu_step_opts_default.restype = None
    L.ntu_trotter_step.argtypes = [vp, i32, tp, tp, tp, ctypes.POINTER(StepOpts), tp]
    L.ntu_profile_enable.argtypes = [vp, i32]
    L.ntu_tune_env.argtypes = [vp, i32, i32, tp, tp, tp, tp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    L.ntu_set_env_ksplit.argtypes = [vp, i32, i32, i32]
    L.ntu_get_env_ksplit.argtypes = [vp, i32, i32]
    L.ntu_set_env_tile.argtypes = [vp, i32, i32, i32]
    L.ntu_get_env_tile.argtypes = [vp, i32, i32]
    L.ntu_tune_save.argtypes = [vp, ctypes.c_char_p]
    L.ntu_tune_load.argtypes = [vp, ctypes.c_char_p]
    L.ntu_profile_read.argtypes = [vp, dp, ctypes.POINTER(i32), i32]
    L.ntu_profile_kind_name.argtypes = [i32]
    L.ntu_profile_kind_name.restype = ctypes.c_char_p
    L.ntu_metric_fix_noalloc.argtypes = [vp, i32, tp, i32, tp]
    L.ntu_superop_gate.argtypes = [vp, i32, tp, tp]
    L.ntu_ctm_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32]
    L.ntu_ctm_destroy.argtypes = [vp]
    L.ntu_ctm_set_stream.argtypes = [vp, vp]
    L.ntu_ctm_last_error.argtypes = [vp]
    L.ntu_ctm_last_error.restype = ctypes.c_char_p
    L.ntu_ctm_run.argtypes = [vp, tp, tp, i32, i32]
    L.ntu_ctm_expect.argtypes = [vp, tp, tp, tp, tp, tp]
    L.ntu_cell_step.argtypes = [vp, i32, i32, tp, i32, ctypes.POINTER(i32), tp, ctypes.POINTER(StepOpts), tp, tp,
                                ctypes.POINTER(i32)]
    L.ntu_evolve.argtypes = [vp, vp, tp, tp, tp, ctypes.POINTER(StepOpts), ctypes.POINTER(EvolveOpts), tp, tp, tp,
                             dp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    for name in EXPORTED:
        if name not in ("ntu_last_error", "ntu_workspace_bytes", "ntu_version", "ntu_fit_opts_default",
                        "ntu_step_opts_default", "ntu_profile_kind_name", "ntu_ctm_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def fit_opts(n_iter=20, early_stop=False, conv_tol=1e-12, kappa=1e-10, ladder=None, tie=1e-15) -> FitOpts:
    o = FitOpts()
    load().ntu_fit_opts_default(ctypes.byref(o))
    o.n_iter, o.early_stop, o.conv_tol, o.kappa, o.tie = n_iter, int(early_stop), conv_tol, kappa, tie
    if ladder is not None:
        o.n_tol = len(ladder)
        for i, t in enumerate(ladder):
            o.tol[i] = t
    return o


def step_opts(precision="f64", fix_mode=FIX_HERM_CLIP, order=(0, 1, 2, 3), scheme="ntu", graph=False,
              **fit) -> StepOpts:
    o = StepOpts()
    load().ntu_step_opts_default(ctypes.byref(o))
    o.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    o.graph = int(graph)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.fix_mode = fix_mode
    o.n_bonds = len(order)
    for i, b in enumerate(order):
        o.order[i] = b
    o.fit = fit_opts(**fit)
    return o


_DTYPES = {torch.float64: F64, torch.complex128: C128, torch.complex64: C64}


def tensor(t):
    """Descriptor of a torch tensor (None -> NULL).  Marshalling only: the
    library checks the element type, shape, strides and memory kind."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dim() > MAX_DIMS:
        raise ValueError(f"at most {MAX_DIMS} dimensions")
    d = Tensor()
    d.data = t.data_ptr()
    d.dtype = _DTYPES.get(t.dtype, -1)
    d.ndim = t.dim()
    for i, (n, st) in enumerate(zip(t.shape, t.stride())):
        d.shape[i], d.stride[i] = n, st
    return d


def _ref(t):
    d = tensor(t)
    return None if d is None else ctypes.byref(d)


class Context:
    """An ``ntu_ctx``: workspace for items up to ``max_D`` and ``max_batch``."""

    def __init__(self, complex_=True, d=2, d_anc=1, r_g=2, max_D=8, max_batch=1, device=0):
        self.L = load()
        self.cplx = complex_
        self.dtype = torch.complex128 if complex_ else torch.float64
        self.d, self.d_anc, self.r_g, self.max_D, self.max_batch = d, d_anc, r_g, max_D, max_batch
        self.p = d * d_anc
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        st = self.L.ntu_ctx_create(ctypes.byref(h), device, C128 if complex_ else F64, d, d_anc, r_g, max_D,
                                   max_batch)
        if st != NTU_OK:
            raise RuntimeError(f"ntu_ctx_create failed ({st}): {self.L.ntu_last_error(None).decode()}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.ntu_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st, what):
        if st != NTU_OK:
            raise RuntimeError(f"{what} failed ({st}): {self.L.ntu_last_error(self.h).decode()}")

    def bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.check(self.L.ntu_set_stream(self.h, ctypes.c_void_p(s)), "ntu_set_stream")

    def set_aux_stream(self, stream=None):
        """Side stream of the Trotter step (a torch.cuda.Stream, or None for
        the context's own)."""
        s = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        self.check(self.L.ntu_set_aux_stream(self.h, s), "ntu_set_aux_stream")

    def empty(self, *shape, dtype=None):
        return torch.empty(*shape, dtype=dtype or self.dtype, device=self.device)

    def zeros(self, *shape, dtype=None):
        return torch.zeros(*shape, dtype=dtype or self.dtype, device=self.device)


def ntu_gate_split(ctx: Context, gate: torch.Tensor):
    """gate: (batch, d^2, d^2) -> GA, GB: (batch, d, d, r_g), sigma: (batch, d^2)."""
    b, d, r = gate.shape[0], ctx.d, ctx.r_g
    GA, GB = ctx.empty(b, d, d, r), ctx.empty(b, d, d, r)
    sig = ctx.empty(b, d * d, dtype=torch.float64)
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_gate_split(ctx.h, b, _ref(gate), _ref(GA), _ref(GB), _ref(sig)), "ntu_gate_split")
    return GA, GB, sig


def ntu_superop_gate(ctx: Context, gate: torch.Tensor):
    """gate: (batch, 4, 4) float64 or complex128 -> S: (batch, 16, 16) float64,
    the action rho -> G rho G^dagger on the Hermitian basis pairs (Eq. 11)."""
    b = gate.shape[0]
    S = torch.empty(b, 16, 16, dtype=torch.float64, device=ctx.device)
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_superop_gate(ctx.h, b, _ref(gate), _ref(S)), "ntu_superop_gate")
    return S


def ntu_reduce_qr(ctx: Context, site: torch.Tensor, gate_factor: torch.Tensor, side: int):
    """site: (batch, p, D, D, D, D); gate_factor: (batch, d, d, r_g) -> Q (batch, pD^3, R), R (batch, R, R)."""
    b, D = site.shape[0], site.shape[2]
    Rd = D * ctx.r_g
    Q, R = ctx.empty(b, ctx.p * D ** 3, Rd), ctx.empty(b, Rd, Rd)
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_reduce_qr(ctx.h, b, _ref(site), _ref(gate_factor), side, _ref(Q), _ref(R)),
              "ntu_reduce_qr")
    return Q, R


def _nbr_array(nbr):
    if len(nbr) != 6:
        raise ValueError("six neighbour tensors expected")
    return (Tensor * 6)(*[tensor(t) for t in nbr])


def ntu_env_contract(ctx: Context, QX, QY, nbr, precision="f64", D=None):
    """QX, QY: (batch, pD^3, R); nbr: six (batch, p, D, D, D, D) -> g (batch, R^2, R^2)."""
    b = QX.shape[0]
    if D is None:
        D = nbr[0].shape[2]
    Rd = D * ctx.r_g
    g = ctx.empty(b, Rd * Rd, Rd * Rd)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_env_contract(ctx.h, b, _ref(QX), _ref(QY), _nbr_array(nbr), prec, _ref(g)),
              "ntu_env_contract")
    return g


def ntu_tune_env(ctx: Context, QX, QY, nbr, precision="bf16x6", D=None, reps=3):
    """Times the metric assembly's schedule candidates (K split; for FP16X3
    also the tile width) on these operands, keeps the fastest in the
    context; -> (K split, mean ms); ntu_get_env_tile gives the width."""
    b = QX.shape[0]
    if D is None:
        D = nbr[0].shape[2]
    Rd = D * ctx.r_g
    g = ctx.empty(b, Rd * Rd, Rd * Rd)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    ks, ms = ctypes.c_int(0), ctypes.c_float(0.0)
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_tune_env(ctx.h, b, prec, _ref(QX), _ref(QY), _nbr_array(nbr), _ref(g), reps,
                                 ctypes.byref(ks), ctypes.byref(ms)), "ntu_tune_env")
    return ks.value, ms.value


def ntu_set_env_ksplit(ctx: Context, D, precision, ks):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    ctx.check(ctx.L.ntu_set_env_ksplit(ctx.h, D, prec, ks), "ntu_set_env_ksplit")


def ntu_get_env_ksplit(ctx: Context, D, precision):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return ctx.L.ntu_get_env_ksplit(ctx.h, D, prec)


def ntu_set_env_tile(ctx: Context, D, precision, width):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    ctx.check(ctx.L.ntu_set_env_tile(ctx.h, D, prec, width), "ntu_set_env_tile")


def ntu_get_env_tile(ctx: Context, D, precision):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return ctx.L.ntu_get_env_tile(ctx.h, D, prec)


def ntu_tune_save(ctx: Context, path):
    ctx.check(ctx.L.ntu_tune_save(ctx.h, str(path).encode()), "ntu_tune_save")


def ntu_tune_load(ctx: Context, path):
    ctx.check(ctx.L.ntu_tune_load(ctx.h, str(path).encode()), "ntu_tune_load")


def ntu_metric_fix(ctx: Context, g: torch.Tensor, D: int | None = None, mode=FIX_HERM_CLIP):
    """In place on g (batch, n, n); returns stats (batch, 8)."""
    b = g.shape[0]
    stats = ctx.zeros(b, 8, dtype=torch.float64)
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_metric_fix(ctx.h, b, _ref(g), mode, _ref(stats)), "ntu_metric_fix")
    return stats


def fit_stats_len(n_iter, D):
    return 16 + 4 * n_iter + D


def ntu_bond_fit(ctx: Context, g, RX, RY, D, opts: FitOpts | None = None):
    """-> MX, MY (batch, R, D), stats (batch, fit_stats_len)."""
    opts = opts or fit_opts()
    b = g.shape[0]
    Rd = D * ctx.r_g
    MX, MY = ctx.empty(b, Rd, D), ctx.empty(b, Rd, D)
    stats = ctx.zeros(b, fit_stats_len(opts.n_iter, D), dtype=torch.float64)
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_bond_fit(ctx.h, b, _ref(g), _ref(RX), _ref(RY), ctypes.byref(opts), _ref(MX), _ref(MY),
                                 _ref(stats)), "ntu_bond_fit")
    return MX, MY, stats


def ntu_recombine(ctx: Context, QX, QY, MX, MY, D):
    b = QX.shape[0]
    Xn, Yn = ctx.empty(b, ctx.p, D, D, D, D), ctx.empty(b, ctx.p, D, D, D, D)
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_recombine(ctx.h, b, _ref(QX), _ref(QY), _ref(MX), _ref(MY), _ref(Xn), _ref(Yn)),
              "ntu_recombine")
    return Xn, Yn


def step_stats_len(n_iter, D):
    return 8 + fit_stats_len(n_iter, D)


def ntu_trotter_step(ctx: Context, A, B, gate_factors, opts: StepOpts | None = None, stats=True):
    """In place on A, B (batch, p, D, D, D, D), compute type or complex64
    storage; gate_factors (batch, 4, 2, d, d, r_g).  Returns stats
    (batch, n_bonds, step_stats_len), a caller's stats tensor when one is
    given, or None."""
    opts = opts or step_opts()
    b, D = A.shape[0], A.shape[2]
    if isinstance(stats, torch.Tensor):
        st = stats
    else:
        st = ctx.zeros(b, opts.n_bonds, step_stats_len(opts.fit.n_iter, D), dtype=torch.float64) if stats else None
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_trotter_step(ctx.h, b, _ref(A), _ref(B), _ref(gate_factors), ctypes.byref(opts), _ref(st)),
              "ntu_trotter_step")
    return st


def ntu_metric_fix_noalloc(g: torch.Tensor, mode=FIX_HERM_CLIP, stats=None):
    """Metric repair without a context or allocation by the library, in
    place on g (batch, n, n) on the current device and torch stream; stats: a
    (batch, 8) float64 tensor or None."""
    L = load()
    s = torch.cuda.current_stream(g.device).cuda_stream
    st = L.ntu_metric_fix_noalloc(ctypes.c_void_p(s), g.shape[0], _ref(g), mode, _ref(stats))
    if st != NTU_OK:
        raise RuntimeError(f"ntu_metric_fix_noalloc failed ({st}): {L.ntu_last_error(None).decode()}")
    return stats


def ntu_profile_enable(ctx: Context, on=True):
    ctx.check(ctx.L.ntu_profile_enable(ctx.h, int(on)), "ntu_profile_enable")


def ntu_profile_read(ctx: Context):
    """-> {kernel class: (total ms, launches)} for the launches recorded since the last read."""
    n = 32
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int * n)()
    k = ctx.L.ntu_profile_read(ctx.h, ms, cnt, n)
    if k < 0:
        raise RuntimeError("ntu_profile_read failed")
    return {ctx.L.ntu_profile_kind_name(i).decode(): (ms[i], cnt[i]) for i in range(k) if cnt[i] > 0}


class CTM:
    """CTMRG environment of a two-site checkerboard state (ntu_ctm_*)."""

    def __init__(self, p, D, chi, device=0):
        self.L = load()
        self.p, self.D, self.chi = p, D, chi
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        st = self.L.ntu_ctm_create(ctypes.byref(h), device, p, D, chi)
        if st != NTU_OK:
            raise RuntimeError(f"ntu_ctm_create: status {st}: {self.L.ntu_last_error(None).decode()}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.ntu_ctm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != NTU_OK:
            raise RuntimeError(f"{what}: status {st}: {self.L.ntu_ctm_last_error(self.h).decode()}")

    def _bind(self):
        self.L.ntu_ctm_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def run(self, A, B, n_iter, reset=True):
        """n_iter iterations for the state (A, B) ((p, D, D, D, D) device tensors)."""
        self._bind()
        self._check(self.L.ntu_ctm_run(self.h, _ref(A), _ref(B), n_iter, int(reset)), "ntu_ctm_run")

    def expect(self, A, B, ops1, ops2):
        """ops1: (n1, p, p), ops2: (n2, 2, p, p) complex128 device tensors ->
        (2 n1 + 4,) complex128: <O_k> at A and B, then <h> on H1, H2, V1, V2."""
        out = torch.empty(2 * ops1.shape[0] + 4, dtype=torch.complex128, device=self.device)
        self._bind()
        self._check(self.L.ntu_ctm_expect(self.h, _ref(A), _ref(B), _ref(ops1), _ref(ops2), _ref(out)),
                    "ntu_ctm_expect")
        return out


def ntu_evolve(ctx: Context, ctm: CTM, A, B, gate_factors, step: StepOpts, n_steps, measure_every, ctm_iters, ops1,
               hb_terms, energy_tol=0.01, ctm_continue=False):
    """An evolution run measured with CTMRG, in place on A, B (1, p, D, D,
    D, D); ops1 (n1, p, p) and hb_terms (n2, 2, p, p) complex128 device
    tensors.  Returns (history (n_meas, 2 n1 + 4) complex128 device tensor,
    energies (n_meas,) numpy, steps taken)."""
    import numpy as np
    max_meas = n_steps // measure_every + 1
    hist = torch.zeros(max_meas, 2 * ops1.shape[0] + 4, dtype=torch.complex128, device=A.device)
    energy = (ctypes.c_double * max_meas)()
    n_meas, steps = ctypes.c_int(0), ctypes.c_int(0)
    ev = EvolveOpts(n_steps, measure_every, ctm_iters, int(ctm_continue), energy_tol)
    ctx.bind_stream()
    st = ctx.L.ntu_evolve(ctx.h, ctm.h, _ref(A), _ref(B), _ref(gate_factors), ctypes.byref(step), ctypes.byref(ev),
                          _ref(ops1), _ref(hb_terms), _ref(hist), energy, ctypes.byref(n_meas), ctypes.byref(steps))
    if st != NTU_OK:
        raise RuntimeError(f"ntu_evolve: status {st}: {ctm.L.ntu_ctm_last_error(ctm.h).decode()} / "
                           f"{ctx.L.ntu_last_error(ctx.h).decode()}")
    k = n_meas.value
    return hist[:k], np.array(energy[:k]), steps.value


CELL_GROUP_MAX = 48


def ntu_cell_step(ctx: Context, Lx, Ly, T, bonds, gate_factors, opts: StepOpts | None = None, stats=True):
    """One sweep of the bonds (x, y, dir) of an Lx x Ly cell, in place on T
    (Lx Ly, p, D, D, D, D); gate_factors (n_bonds, 2, d, d, r_g).  Returns
    (stats (n_bonds, step_stats_len) or None, launch groups)."""
    opts = opts or step_opts()
    n = len(bonds)
    flat = (ctypes.c_int * max(3 * n, 1))(*[int(v) for b in bonds for v in b])
    D = T.shape[2]
    G = min(ctx.max_batch, CELL_GROUP_MAX)
    work = torch.empty(8 * G * T[0].numel(), dtype=T.dtype, device=T.device)
    st = ctx.zeros(n, step_stats_len(opts.fit.n_iter, D), dtype=torch.float64) if stats and n else None
    groups = ctypes.c_int(0)
    ctx.bind_stream()
    ctx.check(ctx.L.ntu_cell_step(ctx.h, Lx, Ly, _ref(T), n, flat, _ref(gate_factors), ctypes.byref(opts), _ref(work),
                                  _ref(st), ctypes.byref(groups)), "ntu_cell_step")
    return st, groups.value
