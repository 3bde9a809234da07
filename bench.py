"""Throughput of the NTU hot path on one MI355X.

Headline ("batched" workload, default --bucket 8): the 48 items of bond
dimension D = 8 of configuration 4 -- independent NTU updates of a
horizontal bond of the 2D transverse-field Ising model, field h_x uniform in
[2.5, 3.5], real-time gate exp(-0.01 i h_b), random complex Gaussian site
tensors drawn as complex64 -- in one batched Trotter-step call per step.
Each update: reduce + QR, environment contraction (split precision on the
matrix cores), metric repair (FP64), bond fit (FP64, <= 20 ALS iterations,
early stop at 1e-12 N), recombination.  The plain FP64 GPU path runs the same
steps from the same state beside it.  ``value`` = bond updates per second of
the split-precision path.

Extra (``mixed_workload``): all 256 items of configuration 4, D uniform in
{3..8}, grouped by D into six buckets, each on its own stream; the buckets
are independent, so the timed region forks them once, runs the K steps of
every bucket back to back and joins them.  --bucket 0 makes this the headline.

"thermal" (configuration 3): imaginary-time evolution of the D = 8 thermal
purification (p = 4, real), one step = one Trotter sweep of 4 bond updates.

"large" (configuration 5): the D = 10 quench state (h_x = 3.04438, dt =
0.005); the whole Trotter sweep is captured once into a HIP graph by the
library (step option graph = 1) and replayed K times (default 1000), on the
split-precision and the FP64 path, each replay followed by a copy of its
statistics into a log, from which the per-step truncation error eps / N of
every bond is reported; the cluster energy of both paths is evaluated every
100 steps (CPU leg).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NTU bond updates/sec at D=8, mixed-precision vs FP64 GPU path, at 1e-6 rel err"
METRIC_HERM = ("NTU bond updates/sec of the manifestly Hermitian purification at D=5 (R=20), split precision "
               "vs FP64 GPU path")
METRIC_SVDU = "SVDU bond updates/sec (reduction, truncated SVD, recombination; no environment)"
PEAK_BF16 = 2.5e15       # dense MFMA, FLOP/s
PEAK_FP64 = 78.6e12      # FLOP/s (vector and matrix)
PEAK_HBM = 8.0e12        # B/s

# The mixed workload runs one stream per bond-dimension bucket (six), each
# with the library's side stream, next to the main stream; HIP maps streams
# onto GPU_MAX_HW_QUEUES hardware queues round-robin (default 4), and streams
# that share a queue serialise.  Ask for enough queues before the runtime
# starts.
HW_QUEUES = 16


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched", choices=["batched", "thermal", "large", "hermitian", "ctmrg", "quench", "cell"])
    ap.add_argument("--precision", default=None, choices=["bf16x3", "bf16x6", "fp16x3", "f64"],
                    help="environment precision (default: fp16x3 for the batched workload; bf16x6 for the "
                         "others, whose real or D > 8 metrics take the tiled path FP16x3 does not cover)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU path")
    ap.add_argument("--scheme", default="ntu", choices=["ntu", "svdu"],
                    help="bond-update scheme: full NTU, or the SVDU update (no environment; implies --no-fp64)")
    ap.add_argument("--e6-tile", type=int, default=0, choices=[0, 128, 256],
                    help="FP16x3: fix the output tile width of the metric assembly after tuning (0: the tuned one)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in K split of the metric assembly instead of autotuning it per bucket")
    ap.add_argument("--bucket", type=int, default=8,
                    help="batched workload: headline on the items of this bond dimension (0 = all 256 items)")
    ap.add_argument("--storage", default="c64", choices=["c64", "c128"],
                    help="batched workload: site tensors stored as complex64 (as drawn) or complex128")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the extra measurement of all 256 items (mixed D)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-roofline", action="store_true",
                    help="skip the K steps timed with per-kernel-class events")
    ap.add_argument("--hw-queues", type=int, default=HW_QUEUES,
                    help="GPU_MAX_HW_QUEUES for this process (hardware queues the streams are spread over)")
    ap.add_argument("--aux", default="own", choices=["own", "shared"],
                    help="side stream of each bucket's Trotter step: the context's own, or one shared by all")
    ap.add_argument("--cell", default="24x24", help="cell workload: Lx x Ly of the unit cell")
    ap.add_argument("--cell-D", type=int, default=8, help="cell workload: bond dimension")
    ap.add_argument("--ctm-D", type=int, default=3,
                    help="bond dimension of the CTMRG and quench workloads (chi = 4 D)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (20 times) and print its "
                         "rate: the reference kernel for scaling HBM byte counters")
    args = ap.parse_args()
    args.steps_given = any(a == "--steps" or a.startswith("--steps=") for a in sys.argv[1:])
    return args


def copy_calibration(mib):
    """A plain copy of known size (read mib MiB, write mib MiB per launch)."""
    import torch
    n = mib * 2 ** 20 // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(20):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / 20
    print(json.dumps({"copy_mib": mib, "bytes_read_per_launch": n * 4, "bytes_written_per_launch": n * 4,
                      "avg_launch_us": ms * 1e3, "rate_GBps": 2 * n * 4 / (ms * 1e-3) / 1e9}))


def fit_flops(R, Dn, half_steps, cg_iters, cplx):
    """Algorithmic FP64 flops of one bond fit on the certified path: per
    half-step g_s = K^H g K and J = K^H g y (R^4 Dn + R^3 Dn^2 + R^3 Dn MACs)
    and cg_iters products with g_s ((R Dn)^2 each); plus g y and the error of
    the guess (2 R^4)."""
    nx = R * Dn
    macs = half_steps * (R ** 4 * Dn + R ** 3 * Dn ** 2 + R ** 3 * Dn + cg_iters * nx ** 2) + 2 * R ** 4
    return macs * (8 if cplx else 2)


def env_work(R, D, p, cplx, fused):
    """Algorithmic work per bond of the environment kernel classes (flops;
    complex multiply-add = 8) and the bytes they must move (FP32 (re, im)
    blocks on the split path).  fused: Right alone, then Left + E4 + E5 in
    one kernel (complex, D^2 <= 64, split precision); otherwise Left and
    Right, E4 and E5 are separate products."""
    m, el = (8, 8) if cplx else (2, 4)
    blk = R * R * D ** 4                      # elements of Left / Right / L2
    q = R * D * D * p * D                     # elements of one dressed isometry
    w = {"env_e6": (m * R ** 4 * D ** 4, 2 * blk * el)}
    if fused:
        w["env_left_right"] = (m * blk * p * D, blk * el + 2 * q * 2 * el)
        w["env_e4"] = (m * (blk * p * D + 2 * R * R * D ** 6), blk * el + 2 * q * 2 * el)
    else:
        w["env_left_right"] = (2 * m * blk * p * D, 2 * blk * el + 4 * q * 2 * el)
        w["env_e4"] = (m * R * R * D ** 6, 2 * blk * el)
        w["env_e5"] = (m * R * R * D ** 6, 2 * blk * el)
    return w


def traffic_record(kernel):
    """HBM bytes per launch of `kernel` from the committed counter runs, or
    None when its source (the kernel's file and the shared headers) has
    changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    srcs = [os.path.join(ROOT, f) for f in rec.get("sources", [rec["source"]])]
    if not all(os.path.exists(f) for f in srcs):
        return None
    if hashlib.sha1(b"".join(open(f, "rb").read() for f in srcs)).hexdigest() != rec["sha1"]:
        return None
    return rec


def host_cpu():
    """CPU model, logical CPUs visible to this process."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    return model, n


class Job:
    """One workload: a list of buckets (one context, stream and batch of items
    each, all of one bond dimension) and the sweep order of a step."""


def bucket_job(ntu, torch, np, dev, items, label, storage):
    buckets = {}
    for it in items:
        buckets.setdefault(it["D"], []).append(it)
    job = Job()
    job.cplx, job.p, job.n_updates, job.items, job.label = True, 2, len(items), items, label
    job.buckets = []
    for D in sorted(buckets):
        its = buckets[D]
        ctx = ntu.Context(complex_=True, d=2, d_anc=1, r_g=2, max_D=D, max_batch=len(its))
        ctx.bind_stream()
        # site tensors stored as drawn (complex64; the step widens them, runs in
        # complex128 and stores the new tensors rounded), or widened once here
        A = torch.from_numpy(np.stack([i["A"] for i in its])).to(dev).to(storage).contiguous()
        B = torch.from_numpy(np.stack([i["B"] for i in its])).to(dev).to(storage).contiguous()
        G = torch.from_numpy(np.stack([i["gate"] for i in its])).to(dev).contiguous()
        GA, GB, _ = ntu.ntu_gate_split(ctx, G)
        gf = torch.zeros(len(its), 4, 2, 2, 2, 2, dtype=torch.complex128, device=dev)
        gf[:, :, 0] = GA[:, None]
        gf[:, :, 1] = GB[:, None]
        job.buckets.append(dict(D=D, A=A, B=B, gf=gf.contiguous(), n=len(its), ctx=ctx,
                                stream=torch.cuda.Stream(device=dev)))
    job.order = (ntu.BOND_H1,)
    job.bonds_per_item = 1
    return job


def thermal_job(ntu, torch, np, dev, inputs, D=8):
    w = inputs.workload_thermal(D=D)
    ctx = ntu.Context(complex_=False, d=2, d_anc=2, r_g=2, max_D=D, max_batch=1)
    ctx.bind_stream()
    G = torch.from_numpy(np.ascontiguousarray(w["gates"][0][None])).to(dev)
    GA, GB, _ = ntu.ntu_gate_split(ctx, G)
    gf = torch.stack([torch.stack([GA[0], GB[0]])] * 4)[None].contiguous()
    A = torch.from_numpy(w["A"][None]).to(dev).contiguous()
    B = torch.from_numpy(w["B"][None]).to(dev).contiguous()
    job = Job()
    job.cplx, job.p, job.n_updates, job.w, job.label = False, 4, 4, w, "thermal"
    job.buckets = [dict(D=D, A=A, B=B, gf=gf, n=1, ctx=ctx, stream=torch.cuda.Stream(device=dev))]
    job.order = (0, 1, 2, 3)
    job.bonds_per_item = 4
    return job


def hermitian_job(ntu, torch, np, dev, inputs, D=5):
    """Manifestly Hermitian purification (Sec. IV): the real iPEPS of rho(beta/2)
    in the basis (X, Y, Z, 1), p = 4, its gate's action on the basis pairs
    formed and split (rank 4, R = 4 D) on the GPU."""
    w = inputs.workload_hermitian_thermal(D=D)
    ctx = ntu.Context(complex_=False, d=4, d_anc=1, r_g=4, max_D=D, max_batch=1)
    ctx.bind_stream()
    G = torch.from_numpy(np.ascontiguousarray(w["gate"][None])).to(dev)
    GA, GB, _ = ntu.ntu_gate_split(ctx, ntu.ntu_superop_gate(ctx, G))
    gf = torch.stack([torch.stack([GA[0], GB[0]])] * 4)[None].contiguous()
    A = torch.from_numpy(w["A"][None]).to(dev).contiguous()
    B = torch.from_numpy(w["B"][None]).to(dev).contiguous()
    job = Job()
    job.cplx, job.p, job.d, job.rg, job.n_updates, job.w, job.label = False, 4, 4, 4, 4, w, "hermitian"
    job.buckets = [dict(D=D, A=A, B=B, gf=gf, n=1, ctx=ctx, stream=torch.cuda.Stream(device=dev))]
    job.order = (0, 1, 2, 3)
    job.bonds_per_item = 4
    return job


def large_job(ntu, torch, np, dev, inputs, D=10):
    w = inputs.workload_large(D=D)
    ctx = ntu.Context(complex_=True, d=2, d_anc=1, r_g=2, max_D=D, max_batch=1)
    ctx.bind_stream()
    G = torch.from_numpy(np.ascontiguousarray(w["gates"][0][None])).to(dev)
    GA, GB, _ = ntu.ntu_gate_split(ctx, G)
    gf = torch.stack([torch.stack([GA[0], GB[0]])] * 4)[None].contiguous()
    A = torch.from_numpy(w["A"][None]).to(dev).contiguous()
    B = torch.from_numpy(w["B"][None]).to(dev).contiguous()
    job = Job()
    job.cplx, job.p, job.n_updates, job.w, job.label = True, 2, 4, w, "large"
    job.buckets = [dict(D=D, A=A, B=B, gf=gf, n=1, ctx=ctx, stream=torch.cuda.Stream(device=dev))]
    job.order = (0, 1, 2, 3)
    job.bonds_per_item = 4
    return job


def run_large(job, args, ntu, torch, np, dev, K):
    """Configuration 5: the captured step replayed K times on each path from
    the seeded state; per-step statistics copied into a log after every
    replay (inside the timed region).  Returns per path: ms per step, the
    logged eps / N of every bond and step, and the states every 100 steps."""
    bk = job.buckets[0]
    ctx, D = bk["ctx"], bk["D"]
    stream = bk["stream"]
    fit = dict(n_iter=20, early_stop=True, conv_tol=1e-12)
    out = {}
    for path in (args.precision, "f64"):
        o = ntu.step_opts(path, order=job.order, graph=True, **fit)
        A, B = bk["A"].clone(), bk["B"].clone()
        st = torch.zeros(1, 4, ntu.step_stats_len(20, D), dtype=torch.float64, device=dev)
        log = torch.zeros(K, 4, dtype=torch.float64, device=dev)
        nsnap = K // 100
        snapA = torch.empty((nsnap,) + tuple(A.shape[1:]), dtype=A.dtype, device=dev)
        snapB = torch.empty_like(snapA)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            # capture + first launch (untimed), then back to the seeded state
            ntu.ntu_trotter_step(ctx, A, B, bk["gf"], o, stats=st)
            A.copy_(bk["A"])
            B.copy_(bk["B"])
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            ev0.record()
            for k in range(K):
                ntu.ntu_trotter_step(ctx, A, B, bk["gf"], o, stats=st)
                log[k].copy_(st[0, :, 8 + 3])          # eps / N of the four bonds
                if (k + 1) % 100 == 0:                 # the state every 100 steps (device copies)
                    snapA[(k + 1) // 100 - 1].copy_(A[0])
                    snapB[(k + 1) // 100 - 1].copy_(B[0])
            ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        snaps = [(100 * (i + 1), snapA[i].cpu().numpy(), snapB[i].cpu().numpy()) for i in range(nsnap)]
        out[path] = {"ms_per_step": ms / K, "log": log.cpu().numpy(), "snaps": snaps}
    return out


class Runner:
    """Warm-up, tuning, timing and per-kernel-class events of one job."""

    def __init__(self, job, args, ntu, torch, dev):
        self.job, self.args, self.ntu, self.torch, self.dev = job, args, ntu, torch, dev
        self.main = torch.cuda.Stream(device=dev)
        self.init = None

    def steps(self, state, o, keep_stats, nsteps):
        """nsteps steps of every bucket.  The buckets are independent: each
        stream waits for the main stream once, runs its nsteps steps back to
        back, and the main stream waits for all of them at the end (main is
        an ordinary stream: work on the legacy null stream would wait for
        every blocking stream of the device)."""
        torch, ntu = self.torch, self.ntu
        main = torch.cuda.current_stream(self.dev)
        assert main.cuda_stream != 0, "run the steps from a non-default stream"
        for bk in self.job.buckets:
            bk["stream"].wait_stream(main)
        out = []
        for _ in range(nsteps):
            st = []
            for bk, (A, B) in zip(self.job.buckets, state):
                with torch.cuda.stream(bk["stream"]):
                    st.append(ntu.ntu_trotter_step(bk["ctx"], A, B, bk["gf"], o, stats=keep_stats))
            out.append(st)
        for bk in self.job.buckets:
            main.wait_stream(bk["stream"])
        return out

    def warm(self, opts64, W):
        """W FP64 steps from the seeded state: both paths start from there."""
        torch = self.torch
        state0 = [(bk["A"].clone(), bk["B"].clone()) for bk in self.job.buckets]
        torch.cuda.synchronize()
        with torch.cuda.stream(self.main):
            self.steps(state0, opts64, False, W)
        torch.cuda.synchronize()
        self.init = state0

    def tune(self, precision):
        """The schedule (K split; FP16x3 also the output tile width) of the
        split-precision metric assembly, per bucket, on
        that bucket's own isometries and neighbours after the warm-up (H1
        cluster: neighbours B, B, B, A, A, A)."""
        torch, ntu = self.torch, self.ntu
        tuning = {}
        with torch.cuda.stream(self.main):
            for bk, (A, B) in zip(self.job.buckets, self.init):
                ctx = bk["ctx"]
                QX, _ = ntu.ntu_reduce_qr(ctx, A, bk["gf"][:, 0, 0].contiguous(), 0)
                QY, _ = ntu.ntu_reduce_qr(ctx, B, bk["gf"][:, 0, 1].contiguous(), 1)
                if self.job.cplx:
                    A, B = A.to(torch.complex128), B.to(torch.complex128)
                ks, tms = ntu.ntu_tune_env(ctx, QX, QY, [B, B, B, A, A, A], precision, D=bk["D"], reps=10)
                rec = {"e6_ksplit": ks, "env_ms": round(tms, 4)}
                if precision == "fp16x3":
                    if self.args.e6_tile:
                        ntu.ntu_set_env_tile(ctx, bk["D"], precision, self.args.e6_tile)
                    rec["e6_tile"] = ntu.ntu_get_env_tile(ctx, bk["D"], precision)
                tuning[str(bk["D"])] = rec
        torch.cuda.synchronize()
        return tuning

    def run(self, o, nsteps, keep_stats=False, profile=False):
        """nsteps steps from the start state between two events on the main
        stream; with profile, the contexts record an event pair around every
        kernel class on their streams."""
        torch, ntu = self.torch, self.ntu
        state = [(A.clone(), B.clone()) for A, B in self.init]
        if profile:
            for bk in self.job.buckets:
                ntu.ntu_profile_enable(bk["ctx"], True)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(self.main):
            ev0.record()
            stats = self.steps(state, o, keep_stats, nsteps)
            ev1.record()
        torch.cuda.synchronize()
        prof = {}
        if profile:
            for bk in self.job.buckets:
                for k, (ms_k, n_k) in ntu.ntu_profile_read(bk["ctx"]).items():
                    a0, b0 = prof.get(k, (0.0, 0))
                    prof[k] = (a0 + ms_k, b0 + n_k)
                ntu.ntu_profile_enable(bk["ctx"], False)
        return ev0.elapsed_time(ev1), state, stats, prof


KERNEL_OF = {"bond_fit": "k_bond_fit_grp (with k_grp_reset, and k_bond_fit for the items it leaves)",
             "env_left_right": "k_right", "env_e4": "k_left_e45",
             "reduce_qr": "k_reduce_cqr_reg (with k_reduce_qr for the items it leaves)", "recombine": "k_recombine",
             "env_e5": "k_mfma_tile (L2)", "env_e6": "k_mfma_tile (g = L2 Right^T)"}


def kernel_of(cls, job, D):
    """Kernel a class runs for a bucket of bond dimension D (the fit's group
    path needs R <= 16 and 5 <= D <= 8; the matrix-core Cholesky QR R <= 16,
    d <= 2 and d^2 r_g <= 32)."""
    rg, d = getattr(job, "rg", 2), getattr(job, "d", 2)
    R = rg * D
    if cls == "bond_fit" and not (R <= 16 and 5 <= D <= 8):
        return "k_bond_fit"
    if cls == "reduce_qr" and not (R <= 16 and d <= 2 and d * d * rg <= 32):
        return ("k_reduce_cholqr (with k_reduce_qr" + ("" if job.cplx else "_reg") +
                " for the items it leaves)")
    return KERNEL_OF[cls]


def rooflines(job, args, stats, nsteps, prof, workload):
    """Per kernel class: algorithmic (and issued MFMA) rate over the average
    launch time of the profiled steps; stats: those steps' stats."""
    import numpy as np
    issue = 1 if args.precision == "f64" else (3 if args.precision in ("bf16x3", "fp16x3") else 6)
    peak_mx = PEAK_FP64 if args.precision == "f64" else PEAK_BF16
    fit_fl, env = 0.0, {}
    for bi, bk in enumerate(job.buckets):
        st = np.stack([x[bi].cpu().numpy() for x in stats])
        R = getattr(job, "rg", 2) * bk["D"]
        for row in st.reshape(-1, st.shape[-1]):
            fit_fl += fit_flops(R, row[8 + 4], 2 * row[8 + 6], row[8 + 15], job.cplx)
        fused = job.cplx and bk["D"] ** 2 <= 64 and args.precision != "f64"
        for k, (fl, by) in env_work(R, bk["D"], job.p, job.cplx, fused).items():
            a0, b0 = env.get(k, (0.0, 0.0))
            env[k] = (a0 + fl * bk["n"] * job.bonds_per_item, b0 + by * bk["n"] * job.bonds_per_item)
    fit_fl /= nsteps                                   # per step
    # HBM classes, algorithmic bytes per step: the reduction reads both site
    # tensors and writes Q and R of both sides; the recombination reads Q and
    # M of both sides and writes both site tensors
    hbm = {"reduce_qr": 0.0, "recombine": 0.0}
    for bk in job.buckets:
        D, R, el = bk["D"], getattr(job, "rg", 2) * bk["D"], 16 if job.cplx else 8
        site, q = job.p * D ** 4, job.p * D ** 3 * R
        nb = bk["n"] * job.bonds_per_item
        hbm["reduce_qr"] += nb * el * 2 * (site + q + R * R)
        hbm["recombine"] += nb * el * 2 * (q + R * D + site)
    rl = {}
    for cls, (t_ms, n_l) in prof.items():
        t = t_ms / nsteps / 1e3                        # s per step
        n_l = n_l / nsteps
        if cls in hbm:
            rl[cls] = {"kernel": kernel_of(cls, job, job.buckets[-1]["D"]), "bound": "hbm", "achieved": hbm[cls] / t / 1e9,
                       "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": hbm[cls] / t / PEAK_HBM,
                       "algorithmic_bytes_per_step": hbm[cls]}
        elif cls == "bond_fit" and args.scheme == "svdu":
            continue
        elif cls == "bond_fit":
            rl[cls] = {"kernel": kernel_of(cls, job, job.buckets[-1]["D"]), "bound": "alu", "achieved": fit_fl / t / 1e12,
                       "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": fit_fl / t / PEAK_FP64,
                       "flops_per_step": fit_fl}
        elif cls in env:
            fl, by = env[cls]
            kern = KERNEL_OF[cls]
            if args.precision == "fp16x3":
                kern = kern.replace("k_mfma_tile ", "k_mfma_tile_f16 ")
            rl[cls] = {"kernel": kern, "bound": "mfma", "achieved": fl / t / 1e12,
                       "peak": peak_mx / 1e12, "unit": "TFLOP/s", "frac": fl / t / peak_mx,
                       "flops_per_step": fl, "issued_mfma_frac": issue * fl / t / peak_mx,
                       "algorithmic_bytes_per_step": by, "algorithmic_GBps": by / t / 1e9}
        else:
            continue
        rl[cls].update({"avg_launch_us": t / n_l * 1e6, "launches_per_step": n_l, "traffic": None})
        rec = traffic_record(rl[cls]["kernel"].split(" ")[0])
        if rec and rec.get("workload") == workload and rec.get("precision") == args.precision:
            rl[cls]["traffic"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
            rl[cls]["traffic_source"] = "profiles/traffic.json"
    dom = max((c for c in prof if c in rl), key=lambda c: prof[c][0], default=None)
    return rl, dom


def fit_summary(job, stats):
    import numpy as np
    its, eig, dmax, phases = {}, 0, 0.0, {}
    for bi, bk in enumerate(job.buckets):
        st = np.stack([s[bi].cpu().numpy() for s in stats])  # steps x items x bonds x len
        its[str(bk["D"])] = float(st[..., 8 + 6].mean())
        eig += int(st[..., 8 + 7].sum())
        dmax = max(dmax, float(st[..., 8 + 3].max()))
        ph = st[..., 8 + 10:8 + 15].reshape(-1, 5).mean(axis=0)
        phases[str(bk["D"])] = {"certificate_kind_mean": float(st[..., 8 + 9].mean()),
                                "cg_iters": float(st[..., 8 + 15].mean()),
                                "kcycles": dict(zip(["setup", "form", "solve", "error", "balance"],
                                                    [round(x / 1e3, 1) for x in ph]))}
    return {"fit_iterations_mean": its, "fit_eig_fallbacks": eig, "delta_max": dmax, "fit_phases": phases}


def measure(job, args, ntu, torch, dev, opts, opts64, K, W, tune=True):
    """Both paths of one job from the same start state: value, FP64 path,
    per-kernel-class rooflines (a second timed pass of K steps with events
    around every kernel class)."""
    r = Runner(job, args, ntu, torch, dev)
    r.warm(opts64, W)
    out = {}
    if tune and args.precision in ("bf16x3", "bf16x6", "fp16x3") and not args.no_tune and args.scheme == "ntu":
        out["tuning"] = r.tune(args.precision)
    # one untimed step of the measured path, so that no kernel of it is
    # launched for the first time inside the timed region
    r.run(opts, 1)
    ms, state, stats, _ = r.run(opts, K, keep_stats=True)
    upd = job.n_updates
    out.update({"value": upd * K / (ms / 1e3), "ms_per_step": ms / K, "state": state, "stats": stats})
    if not args.no_fp64:
        r.run(opts64, 1)
        ms64, _, _, _ = r.run(opts64, K)
        out["fp64_path"] = {"value": upd * K / (ms64 / 1e3), "ms_per_step": ms64 / K}
        out["speedup_vs_fp64_path"] = out["value"] / out["fp64_path"]["value"]
    if not args.no_roofline:
        msp, _, stp, prof = r.run(opts, K, keep_stats=True, profile=True)
        out["prof"], out["prof_stats"], out["ms_per_step_with_kernel_events"] = prof, stp, msp / K
    out["runner"] = r
    return out


def metric_sample(job, ntu, torch, precision, n_items=2):
    """Metric of the first items of the first bucket, from the seeded state
    (H1 cluster), on both GPU paths: for comparison with the oracle."""
    bk = job.buckets[0]
    ctx = bk["ctx"]
    ctx.bind_stream()
    A = bk["A"][:n_items].to(torch.complex128).contiguous()
    B = bk["B"][:n_items].to(torch.complex128).contiguous()
    QX, _ = ntu.ntu_reduce_qr(ctx, A, bk["gf"][:n_items, 0, 0].contiguous(), 0)
    QY, _ = ntu.ntu_reduce_qr(ctx, B, bk["gf"][:n_items, 0, 1].contiguous(), 1)
    nb = [B, B, B, A, A, A]
    g64 = ntu.ntu_env_contract(ctx, QX, QY, nb, "f64", D=bk["D"])
    gmx = ntu.ntu_env_contract(ctx, QX, QY, nb, precision, D=bk["D"])
    torch.cuda.synchronize()
    return g64.cpu().numpy(), gmx.cpu().numpy()


def main_large(args, ntu, torch, np, dev, inputs):
    """Configuration 5 (see the module docstring)."""
    K = args.steps if args.steps_given else 1000
    job = large_job(ntu, torch, np, dev, inputs)
    res = run_large(job, args, ntu, torch, np, dev, K)
    mx, f64 = res[args.precision], res["f64"]
    result = {
        "metric": METRIC, "value": 4 / (mx["ms_per_step"] / 1e3), "unit": "bond_updates/s", "n_gpus": 1,
        "steps": K, "warmup": 0, "ms_per_step": mx["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"{args.precision}+f64", "data": "synthetic",
        "config": {"workload": "configuration 5: D=10 quench (h_x=3.04438, dt=0.005), 2-site unit cell, "
                               "whole Trotter step captured in a HIP graph by the library and replayed",
                   "D": 10, "replays": K, "env_precision": args.precision,
                   "fit": "fp64, <=20 ALS iterations, early stop 1e-12 N", "bond_updates_per_step": 4,
                   "start": "seeded random state", "logging": "eps/N of every bond copied after every replay"},
        "fp64_path": {"value": 4 / (f64["ms_per_step"] / 1e3), "ms_per_step": f64["ms_per_step"]},
        "speedup_vs_fp64_path": f64["ms_per_step"] / mx["ms_per_step"],
        "truncation_error": {p: {"mean": float(r["log"].mean()), "max": float(r["log"].max()),
                                 "final_step": [float(x) for x in r["log"][-1]]}
                             for p, r in ((args.precision, mx), ("f64", f64))},
    }
    if not args.no_cpu:
        from oracle import ntu as O
        t0 = time.perf_counter()
        drift = []
        e0, _ = O.observables(job.w["A"], job.w["B"], inputs.H_CRIT)
        for (k, A1, B1), (_, A2, B2) in zip(mx["snaps"], f64["snaps"]):
            e1, x1 = O.observables(A1, B1, inputs.H_CRIT)
            e2, x2 = O.observables(A2, B2, inputs.H_CRIT)
            drift.append({"step": k, "energy": e2, "energy_split_minus_fp64": e1 - e2, "sx_split_minus_fp64": x1 - x2})
        result["energy_drift"] = {"initial_energy": e0, "samples": drift,
                                  "estimator": "cluster estimator of the oracle (CPU)"}
        result["energy_drift_cpu_seconds"] = time.perf_counter() - t0
    print(json.dumps(result), flush=True)


def main_ctmrg(args, ntu, torch, np, dev, inputs):
    """CTMRG expectation values (the environment the paper uses for
    observables, chi = 4 D as in Sec. III) of a configuration-2 quench state
    evolved on the GPU; K iterations timed after W untimed ones."""
    D = args.ctm_D
    chi = 4 * D
    K = args.steps if args.steps_given else 20
    W = args.warmup
    w = inputs.workload_quench(seed=2, D=D)
    ctx = ntu.Context(complex_=True, d=2, d_anc=1, r_g=2, max_D=D, max_batch=1)
    ctx.bind_stream()
    G = torch.from_numpy(np.ascontiguousarray(w["gates"][0][None])).to(dev)
    GA, GB, _ = ntu.ntu_gate_split(ctx, G)
    gf = torch.stack([torch.stack([GA[0], GB[0]])] * 4)[None].contiguous()
    A = torch.from_numpy(w["A"][None]).to(dev).contiguous()
    B = torch.from_numpy(w["B"][None]).to(dev).contiguous()
    o64 = ntu.step_opts("f64", n_iter=20, early_stop=True, conv_tol=1e-12)
    for _ in range(5):
        ntu.ntu_trotter_step(ctx, A, B, gf, o64)
    torch.cuda.synchronize()
    A0, B0 = A[0].contiguous(), B[0].contiguous()
    ctm = ntu.CTM(2, D, chi)
    ctm.run(A0, B0, max(W, 1))
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ctm.run(A0, B0, K, reset=True)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    X = np.array([[0, 1], [1, 0]], complex)
    Z = np.diag([1.0, -1.0]).astype(complex)
    ops1 = torch.from_numpy(np.stack([X, Z])).to(dev)
    ops2 = torch.from_numpy(np.stack([np.stack([Z, Z])])).to(dev)
    t0 = time.perf_counter()
    vals = ctm.expect(A0, B0, ops1, ops2).cpu().numpy()
    t_exp = time.perf_counter() - t0
    hx = inputs.H_CRIT
    sx = 0.5 * (vals[0] + vals[1]).real
    e = float(-0.5 * vals[4:8].sum().real - hx * sx)
    result = {
        "metric": f"CTMRG iterations/s at chi=4D (D={D})", "value": K / (ms / 1e3), "unit": "iterations/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"CTMRG environment of a configuration-2 quench state (seed 2, D={D}, five FP64 NTU "
                               f"sweeps at dt=0.01 on the GPU), chi={chi}, 2x2 cell, four directional moves per "
                               f"iteration, from the identity boundary", "D": D, "chi": chi},
        "observables": {"energy_per_site": e, "sx": sx, "expect_seconds": t_exp,
                        "after_iterations": K},
    }
    if not args.no_cpu:
        from oracle import ctmrg as OC
        An, Bn = A0.cpu().numpy(), B0.cpu().numpy()
        t0 = time.perf_counter()
        n = 0
        env = None
        while time.perf_counter() - t0 < args.cpu_seconds:
            env = OC.ctmrg(An, Bn, chi, 1, env=env)
            n += 1
        el = time.perf_counter() - t0
        model, ncpu = host_cpu()
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        result["cpu_baseline"] = {"value": n / el, "unit": "iterations/s", "cores": cores, "kind": "oracle",
                                  "sample": f"{n} CTMRG iterations of the same state from the identity boundary, "
                                            f"oracle FP64 numpy/BLAS", "cpu_model": model,
                                  "logical_cpus_visible": ncpu}
    print(json.dumps(result), flush=True)


def main_quench(args, ntu, torch, np, dev, inputs):
    """The quench run of Sec. III through ntu_evolve: from |+> at h_x = h_c,
    second-order sweeps of half-step gates at dt = 0.01 (the paper's step),
    FP64, a CTMRG measurement (chi = 4 D, 15 iterations continued from the
    previous environment) every 10 steps and the 0.01 energy stop; K steps
    timed (default 40) after W untimed ones."""
    D = args.ctm_D
    chi = 4 * D
    K = args.steps if args.steps_given else 40
    W = args.warmup
    dt, hx, every, iters = 0.01, inputs.H_CRIT, 10, 15
    order = ["H1", "H2", "V1", "V2", "V2", "V1", "H2", "H1"]
    codes = dict(H1=ntu.BOND_H1, H2=ntu.BOND_H2, V1=ntu.BOND_V1, V2=ntu.BOND_V2)
    ctx = ntu.Context(complex_=True, d=2, d_anc=1, r_g=2, max_D=D, max_batch=1)
    ctx.bind_stream()
    Gh = torch.from_numpy(inputs.bond_gate(inputs.ising_bond_hamiltonian(hx), dt / 2)[None]).to(dev)
    GA, GB, _ = ntu.ntu_gate_split(ctx, Gh)
    gf = torch.stack([torch.stack([GA[0], GB[0]])] * 4)[None].contiguous()
    step = ntu.step_opts("f64", order=[codes[b] for b in order], n_iter=20, early_stop=True, conv_tol=1e-12)
    X = np.array([[0, 1], [1, 0]], complex)
    Zm = np.diag([1.0, -1.0]).astype(complex)
    hb = inputs.ising_bond_hamiltonian(hx)
    # h_b = -ZZ - (h_x / 4)(X 1 + 1 X) as a sum of products
    I2 = np.eye(2, dtype=complex)
    terms = np.stack([np.stack([-Zm, Zm]), np.stack([-0.25 * hx * X, I2]), np.stack([I2, -0.25 * hx * X])])
    assert np.abs(sum(np.kron(a, b) for a, b in terms) - hb).max() < 1e-14
    ops1 = torch.from_numpy(np.stack([X, Zm])).to(dev)
    hbt = torch.from_numpy(terms).to(dev)
    A0, B0 = inputs.polarised_x(D)
    ctm = ntu.CTM(2, D, chi)
    if W:
        A = torch.from_numpy(A0[None]).to(dev)
        B = torch.from_numpy(B0[None]).to(dev)
        ntu.ntu_evolve(ctx, ctm, A, B, gf, step, W, every, iters, ops1, hbt, 0.01, True)
    A = torch.from_numpy(A0[None]).to(dev)
    B = torch.from_numpy(B0[None]).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, e, steps = ntu.ntu_evolve(ctx, ctm, A, B, gf, step, K, every, iters, ops1, hbt, 0.01, True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h = hist.cpu().numpy()
    result = {
        "metric": f"quench run: Trotter steps/s with CTMRG measurements (D={D}, chi={chi})",
        "value": steps / el, "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": W,
        "ms_per_step": 1e3 * el / max(steps, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"Sec. III quench from |+> at h_x=3.04438, D={D}, second-order sweeps of half-step "
                               f"gates at dt=0.01, FP64, CTMRG chi={chi} ({iters} iterations continued) every "
                               f"{every} steps, 0.01 energy stop", "D": D, "chi": chi},
        "observables": {"t": [round(k * every * dt, 4) for k in range(len(e))], "energy": [float(v) for v in e],
                        "sx": [float(0.5 * (r[0] + r[1]).real) for r in h], "steps_done": steps},
    }
    if not args.no_cpu:
        from oracle import evolve as OE
        from oracle import ntu as ON
        GAo, GBo, _ = ON.gate_split(inputs.bond_gate(hb, dt / 2), 2, 2)
        gd = {b: (GAo, GBo) for b in ON.BONDS}
        # the oracle's cost of one step and of one measurement, composed into
        # the GPU run's schedule (K steps, a measurement before them and one
        # every `every` steps)
        t0 = time.perf_counter()
        env, _ = OE.measure(A0, B0, chi, iters, [X, Zm], hb)
        t_meas = time.perf_counter() - t0
        An, Bn = A0, B0
        n_cpu = 2
        t0 = time.perf_counter()
        for _ in range(n_cpu):
            An, Bn, _ = ON.trotter_step(An, Bn, gd, D, n_iter=20, conv_tol=1e-12, order=order)
        t_step = (time.perf_counter() - t0) / n_cpu
        n_meas = steps // every + 1
        model, ncpu = host_cpu()
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        result["cpu_baseline"] = {"value": steps / (steps * t_step + n_meas * t_meas), "unit": "steps/s",
                                  "cores": cores, "kind": "oracle",
                                  "sample": f"oracle: one measurement ({t_meas:.2f} s, {iters} CTMRG iterations "
                                            f"from the identity boundary) and {n_cpu} second-order steps "
                                            f"({t_step:.2f} s each) of the same run, composed into the GPU run's "
                                            f"{steps} steps and {n_meas} measurements",
                                  "cpu_model": model, "logical_cpus_visible": ncpu}
    ctm.close()
    print(json.dumps(result), flush=True)


def main_cell(args, ntu, torch, np, dev, inputs):
    """One sweep over every bond of an Lx x Ly unit cell of distinct random
    complex tensors (ntu_cell_step, the library's sweep order; the quench
    gate at dt = 0.01 on every bond): bond updates/s in the chosen precision
    and in FP64, K sweeps timed (default 5) after W untimed ones."""
    Lx, Ly = (int(v) for v in args.cell.lower().split("x"))
    D = args.cell_D
    K = args.steps if args.steps_given else 5
    W = args.warmup
    rng = np.random.default_rng(6)
    sites = np.stack([inputs.random_site_pair(rng, 2, D)[0] for _ in range(Lx * Ly)])
    bonds = inputs.cell_bond_order(Lx, Ly)
    G = inputs.bond_gate(inputs.ising_bond_hamiltonian(inputs.H_CRIT), 0.01)
    ctx = ntu.Context(complex_=True, d=2, d_anc=1, r_g=2, max_D=D, max_batch=48)
    ctx.bind_stream()
    GA, GB, _ = ntu.ntu_gate_split(ctx, torch.from_numpy(G[None]).to(dev))
    gf = torch.stack([GA[0], GB[0]])[None].expand(len(bonds), 2, *GA.shape[1:]).contiguous()
    out = {}
    for prec in (args.precision, "f64"):
        T = torch.from_numpy(sites).to(dev)
        opts = ntu.step_opts(prec, n_iter=20, early_stop=True, conv_tol=1e-12)
        for _ in range(W):
            ntu.ntu_cell_step(ctx, Lx, Ly, T, bonds, gf, opts, stats=False)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n = K if prec == args.precision else max(1, min(K, 2))
        ev0.record()
        groups = 0
        for _ in range(n):
            _, groups = ntu.ntu_cell_step(ctx, Lx, Ly, T, bonds, gf, opts, stats=False)
        ev1.record()
        torch.cuda.synchronize()
        out[prec] = (ev0.elapsed_time(ev1) / n, groups)
    ms, groups = out[args.precision]
    ms64 = out["f64"][0]
    nb = len(bonds)
    result = {
        "metric": f"NTU bond updates/s over a {Lx}x{Ly} unit cell at D={D}", "value": nb / (ms / 1e3),
        "unit": "bond_updates/s", "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{Lx}x{Ly} unit cell of distinct random complex site tensors (seed 6), D={D}, "
                               f"one sweep of its {nb} bonds (critical quench gate, dt=0.01) per step in "
                               f"{groups} launch groups of independent bonds", "D": D, "bonds": nb,
                   "groups": groups},
        "fp64_path": {"value": nb / (ms64 / 1e3), "ms_per_step": ms64},
    }
    if not args.no_cpu:
        from oracle import cell as OCE
        from oracle import ntu as ON
        GAo, GBo, _ = ON.gate_split(G, 2, 2)
        T0 = {(k % Lx, k // Lx): sites[k] for k in range(Lx * Ly)}
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < args.cpu_seconds and done < nb:
            k = min(8, nb - done)
            T0, _ = OCE.cell_sweep(T0, Lx, Ly, bonds[done:done + k], [(GAo, GBo)] * k, D, n_iter=20,
                                   conv_tol=1e-12)
            done += k
        el = time.perf_counter() - t0
        model, ncpu = host_cpu()
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        result["cpu_baseline"] = {"value": done / el, "unit": "bond_updates/s", "cores": cores, "kind": "oracle",
                                  "sample": f"the first {done} bond updates of the same sweep, oracle FP64 "
                                            f"numpy/BLAS", "cpu_model": model, "logical_cpus_visible": ncpu}
    print(json.dumps(result), flush=True)


def run_mixed_child(args, K, W):
    """The mixed workload (--bucket 0) in a child process; its JSON line
    reduced to the fields reported under mixed_workload."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--bucket", "0", "--no-cpu", "--no-roofline",
           "--steps", str(K), "--warmup", str(W), "--precision", args.precision, "--storage", args.storage,
           "--hw-queues", str(args.hw_queues), "--aux", args.aux]
    for flag in ("no_fp64", "no_tune"):
        if getattr(args, flag):
            cmd.append("--" + flag.replace("_", "-"))
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=900)
    if out.returncode != 0:
        raise RuntimeError("mixed workload run failed:\n" + out.stderr[-4000:])
    mm = json.loads(out.stdout.strip().splitlines()[-1])
    mixed = {"workload": mm["config"]["workload"], "items": mm["config"]["items"], "value": mm["value"],
             "unit": "bond_updates/s", "ms_per_step": mm["ms_per_step"], "D_counts": mm["config"].get("D_counts"),
             "streams": mm["config"].get("streams"), "process": "child process, run before this one uses the GPU"}
    for k in ("fp64_path", "speedup_vs_fp64_path", "tuning"):
        if k in mm:
            mixed[k] = mm[k]
    return mixed


def main():
    args = parse()
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the bond updates of a step are "
              "independent, and the multi-GPU layout is described but not run", file=sys.stderr)
        sys.exit(2)
    if args.copy_mib:
        copy_calibration(args.copy_mib)
        return
    K, W = args.steps, args.warmup
    if args.precision is None:
        args.precision = ("fp16x3" if args.workload == "batched" or (args.workload == "cell" and args.cell_D <= 8)
                          else "bf16x6")
    # extra: all 256 items of configuration 4 (mixed D), measured first, in a
    # child process, before this process touches the GPU: its thirteen
    # streams then have the hardware queues to themselves
    mixed_result = None
    if args.workload == "batched" and args.bucket and not args.no_mixed and args.scheme == "ntu":
        mixed_result = run_mixed_child(args, K, W)
    import numpy as np
    import torch
    from paper_2107_06635_amd import inputs
    from paper_2107_06635_amd import ntu

    dev = torch.device("cuda", 0)
    if args.scheme == "svdu":
        args.no_fp64 = True
    if args.workload == "large":
        main_large(args, ntu, torch, np, dev, inputs)
        return
    if args.workload == "ctmrg":
        main_ctmrg(args, ntu, torch, np, dev, inputs)
        return
    if args.workload == "quench":
        main_quench(args, ntu, torch, np, dev, inputs)
        return
    if args.workload == "cell":
        main_cell(args, ntu, torch, np, dev, inputs)
        return
    all_items = None
    if args.workload == "batched":
        all_items = inputs.workload_batched()
        if args.bucket:
            items = [it for it in all_items if it["D"] == args.bucket]
            label = (f"configuration 4, its {len(items)} D={args.bucket} items: independent H1 bond updates, "
                     f"one batched call per step")
        else:
            items, label = all_items, "configuration 4: 256 independent bond updates, D uniform in {3..8}"
        storage = torch.complex64 if args.storage == "c64" else torch.complex128
        job = bucket_job(ntu, torch, np, dev, items, label, storage)
    elif args.workload == "hermitian":
        job = hermitian_job(ntu, torch, np, dev, inputs)
    else:
        job = thermal_job(ntu, torch, np, dev, inputs)
    if args.aux == "shared":
        job.aux = torch.cuda.Stream(device=dev)
        for bk in job.buckets:
            bk["ctx"].set_aux_stream(job.aux)
    fit = dict(n_iter=20, early_stop=True, conv_tol=1e-12)
    opts = ntu.step_opts(args.precision, order=job.order, scheme=args.scheme, **fit)
    opts64 = ntu.step_opts("f64", order=job.order, **fit)

    m = measure(job, args, ntu, torch, dev, opts, opts64, K, W)
    result = {
        "metric": (METRIC_SVDU if args.scheme != "ntu" else METRIC_HERM if args.workload == "hermitian"
                   else METRIC),
        "value": m["value"],
        "unit": "bond_updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.precision}+f64",
        "data": "synthetic",
    }
    if args.workload == "batched":
        result["config"] = {"workload": job.label, "items": job.n_updates,
                            "D_counts": {str(bk["D"]): bk["n"] for bk in job.buckets},
                            "h_x": "uniform [2.5, 3.5]", "dt": 0.01, "env_precision": args.precision,
                            "fit": ("fp64, <=20 ALS iterations, early stop 1e-12 N" if args.scheme == "ntu"
                                    else "none (SVDU scheme)"),
                            "scheme": args.scheme,
                            "storage": ("site tensors stored in complex64 (widened at the start of each step, "
                                        "written back rounded), step computed in complex128"
                                        if args.storage == "c64" else
                                        "values drawn as complex64, widened once, stored in complex128"),
                            "start": f"seeded state + {W} FP64 warm-up steps"}
        if len(job.buckets) > 1:
            result["config"]["streams"] = (f"one per D bucket, side streams "
                                           f"{'one shared' if args.aux == 'shared' else 'one per bucket'}, "
                                           f"{args.hw_queues} hardware queues")
    elif args.workload == "hermitian":
        w = job.w
        result["config"] = {"workload": "manifestly Hermitian purification (Sec. IV): one state, D=5, "
                                        "p=d^2=4, real, gate action of rank 4 (R=20)", "D": w["D"],
                            "h_x": w["hx"], "h_z": w["hz"], "dbeta": w["dbeta"], "env_precision": args.precision,
                            "fit": "fp64, <=20 ALS iterations, early stop 1e-12 N", "bond_updates_per_step": 4,
                            "start": f"rho(0/2) = 1 + {W} FP64 warm-up steps"}
    else:
        result["config"] = {"workload": "configuration 3: thermal purification, D=8, p=4, real", "D": 8,
                            "h_x": 2.5, "dbeta": 0.005, "env_precision": args.precision,
                            "fit": "fp64, <=20 ALS iterations, early stop 1e-12 N", "bond_updates_per_step": 4,
                            "start": f"beta=0 purification + {W} FP64 warm-up steps"}
    if "tuning" in m:
        result["tuning"] = m["tuning"]
    if "fp64_path" in m:
        result["fp64_path"] = m["fp64_path"]
        result["speedup_vs_fp64_path"] = m["speedup_vs_fp64_path"]
    result.update(fit_summary(job, m["stats"]))
    if "prof" in m:
        prof = m["prof"]
        result["ms_per_step_with_kernel_events"] = m["ms_per_step_with_kernel_events"]
        result["kernel_ms_per_step"] = {k: round(v[0] / K, 4) for k, v in
                                        sorted(prof.items(), key=lambda kv: -kv[1][0])}
        rl, dom = rooflines(job, args, m["prof_stats"], K, prof, job.label)
        result["roofline"] = dict(rl.get(dom, {}), dominant_class=dom)
        result["roofline_by_class"] = rl

    # metric of the first items from the seeded state, both GPU paths (the
    # oracle's comparison is made in the CPU leg below)
    gs = None
    if args.workload == "batched" and args.scheme == "ntu" and args.precision != "f64":
        gs = metric_sample(job, ntu, torch, args.precision)
        g64, gmx = gs
        errs = [float(np.linalg.norm(gmx[i] - g64[i]) / np.linalg.norm(g64[i])) for i in range(len(g64))]
        result["metric_rel_err_vs_fp64_path"] = {"D": job.buckets[0]["D"], "items": len(errs), "max": max(errs)}

    if mixed_result is not None:
        result["mixed_workload"] = mixed_result

    if not args.no_cpu:
        from oracle import ntu as O
        t0 = time.perf_counter()
        n_bonds = 0
        g_oracle = []
        if args.workload == "batched":
            # the headline items in order, cycling until the time budget is spent
            while time.perf_counter() - t0 < args.cpu_seconds:
                it = job.items[n_bonds % len(job.items)]
                GAo, GBo, _ = O.gate_split(it["gate"], 2, 2)
                A = it["A"].astype(np.complex128)
                B = it["B"].astype(np.complex128)
                X, Y, nbr = O._cluster(True, A, B)
                if args.scheme == "svdu":
                    O.svdu_update(X, Y, GAo, GBo, it["D"])
                else:
                    _, _, info = O.bond_update(X, Y, nbr, GAo, GBo, it["D"], n_iter=20, conv_tol=1e-12)
                    if gs is not None and n_bonds < len(gs[0]):
                        g_oracle.append(info["g_raw"])
                n_bonds += 1
            sample = (f"{n_bonds} bond updates cycling in order through the {len(job.items)} items of the headline "
                      f"workload from their seeded state, oracle FP64 numpy/BLAS"
                      f"{', SVDU updates' if args.scheme == 'svdu' else ''}")
        elif args.workload == "hermitian":
            from oracle import hermitian as OH
            r = m["runner"]
            An, Bn = r.init[0][0].cpu().numpy()[0], r.init[0][1].cpu().numpy()[0]
            D = job.buckets[0]["D"]
            GAo, GBo, _ = OH.gate_factors(job.w["gate"])
            pairs = {b: (GAo, GBo) for b in O.BONDS}
            while n_bonds < 64 and time.perf_counter() - t0 < args.cpu_seconds:
                for b in O.BONDS:
                    An, Bn, _ = O.trotter_step(An, Bn, pairs, D, d=4, n_iter=20, conv_tol=1e-12, order=(b,),
                                                scheme=args.scheme)
                    n_bonds += 1
            sample = (f"{n_bonds} bond updates of the D={D} Hermitian purification from the warmed-up state, "
                      f"oracle FP64 numpy/BLAS")
        else:
            r = m["runner"]
            An, Bn = r.init[0][0].cpu().numpy()[0], r.init[0][1].cpu().numpy()[0]
            GAo, GBo, _ = O.gate_split(job.w["gates"][0], 2, 2)
            pairs = {b: (GAo, GBo) for b in O.BONDS}
            while n_bonds < 16 and time.perf_counter() - t0 < args.cpu_seconds:
                for b in O.BONDS:
                    An, Bn, _ = O.trotter_step(An, Bn, pairs, 8, n_iter=20, conv_tol=1e-12, order=(b,),
                                                scheme=args.scheme)
                    n_bonds += 1
            sample = f"{n_bonds} bond updates of the D=8 thermal state, oracle FP64 numpy/BLAS"
        el = time.perf_counter() - t0
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        model, ncpu = host_cpu()
        result["cpu_baseline"] = {"value": n_bonds / el, "unit": "bond_updates/s", "cores": cores, "kind": "oracle",
                                  "sample": sample, "cpu_model": model, "logical_cpus_visible": ncpu}
        if g_oracle:
            g64, gmx = gs
            k = len(g_oracle)
            e_mx = [float(np.linalg.norm(gmx[i] - g_oracle[i]) / np.linalg.norm(g_oracle[i])) for i in range(k)]
            e_64 = [float(np.linalg.norm(g64[i] - g_oracle[i]) / np.linalg.norm(g_oracle[i])) for i in range(k)]
            result["metric_rel_err_vs_oracle"] = {"D": job.buckets[0]["D"], "items": k, "precision": args.precision,
                                                  "max": max(e_mx), "fp64_path_max": max(e_64),
                                                  "state": "seeded state, H1 cluster"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
