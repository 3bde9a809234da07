"""Throughput of the NTU hot path on one MI355X.

Workload (default): imaginary-time evolution of the thermal purification of
the 2D transverse-field Ising model, D = 8, physical d = 2 plus ancilla d = 2
(p = 4), real arithmetic, gate exp(-0.005 h_b) at h_x = 2.5, from the beta = 0
product purification.  One step = one first-order Trotter sweep = 4 NTU bond
updates (H1, H2, V1, V2), each: reduce + QR, environment contraction (split
precision on MFMA), metric repair (FP64), bond fit (FP64, <= 20 ALS
iterations, early stop at 1e-12 N), recombination.

Prints ONE JSON line.  ``value`` = bond updates per second of the mixed path;
the plain FP64 GPU path runs the same steps from the same state beside it.
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
PEAK_BF16 = 2.5e15       # dense MFMA, FLOP/s
PEAK_FP64 = 78.6e12      # FLOP/s (vector and matrix)
PEAK_HBM = 8.0e12        # B/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--D", type=int, default=8)
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "bf16x6", "f64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--profile-steps", type=int, default=2)
    return ap.parse_args()


def fit_flops_per_launch(R, Dn, half_steps, cplx):
    """Algorithmic FP64 flops of one bond-fit launch (certified solves):
    per half-step g_s = K^H g K (R^4 Dn + R^3 Dn^2 MACs), Cholesky (nx^3/3),
    triangular inverse (nx^3/6), two triangular mat-vecs (nx^2), error
    d^H g d (R^4); plus the SVDU / balancing products."""
    nx = R * Dn
    macs = half_steps * (R ** 4 * Dn + R ** 3 * Dn ** 2 + nx ** 3 / 2 + nx ** 2 + R ** 4)
    macs += 3 * R ** 4   # g y, SVDU error, balancing product
    return macs * (8 if cplx else 2)


def e6_flops(R, D, cplx):
    return (8 if cplx else 2) * (R * R) * (R * R) * D ** 4


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); a multi-GPU run is not part of this build",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2107_06635_amd import inputs
    from paper_2107_06635_amd import ntu

    dev = torch.device("cuda", 0)
    D, K, W = args.D, args.steps, args.warmup
    w = inputs.workload_thermal(D=D)
    ctx = ntu.Context(complex_=False, d=2, d_anc=2, r_g=2, max_D=D, max_batch=1)
    ctx.bind_stream()
    # gate factors on the GPU (the same gate on all four bonds)
    G = torch.from_numpy(np.ascontiguousarray(w["gates"][0][None])).to(dev)
    GA, GB, _ = ntu.ntu_gate_split(ctx, G)
    gf = torch.stack([torch.stack([GA[0], GB[0]])] * 4)[None].contiguous()
    A = torch.from_numpy(w["A"][None]).to(dev).contiguous()
    B = torch.from_numpy(w["B"][None]).to(dev).contiguous()
    fit = dict(n_iter=20, early_stop=True, conv_tol=1e-12)
    opts = ntu.step_opts(args.precision, **fit)
    opts64 = ntu.step_opts("f64", **fit)

    # warm-up from beta = 0 on the FP64 path, so both paths start from the same state
    for _ in range(W):
        ntu.ntu_trotter_step(ctx, A, B, gf, opts64, stats=False)
    torch.cuda.synchronize()
    A0, B0 = A.clone(), B.clone()

    def run(o, steps, keep_stats=False):
        Aw, Bw = A0.clone(), B0.clone()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stats = []
        ev0.record()
        for _ in range(steps):
            st = ntu.ntu_trotter_step(ctx, Aw, Bw, gf, o, stats=keep_stats)
            if keep_stats:
                stats.append(st)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1), Aw, Bw, stats

    ms, Am, Bm, stm = run(opts, K, keep_stats=True)
    result = {
        "metric": METRIC,
        "value": 4 * K / (ms / 1e3),
        "unit": "bond_updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.precision}+f64",
        "data": "synthetic",
        "config": {"workload": "thermal purification (configuration 3), D=8", "D": D, "p": 4, "d": 2, "d_anc": 2,
                   "h_x": 2.5, "dbeta": 0.005, "env_precision": args.precision,
                   "fit": "fp64, <=20 ALS iterations, early stop 1e-12 N", "bond_updates_per_step": 4,
                   "start": f"beta=0 purification + {W} FP64 warm-up steps"},
    }
    st_all = torch.stack(stm).cpu().numpy()[:, 0]          # steps x bonds x len
    fl = ntu.fit_stats_len(20, D)
    iters = st_all[:, :, 8 + 6]
    dn = st_all[:, :, 8 + 4]
    result["fit_iterations_mean"] = float(iters.mean())
    result["fit_eig_fallbacks"] = int(st_all[:, :, 8 + 7].sum())
    result["delta_max"] = float(st_all[:, :, 8 + 3].max())

    if not args.no_fp64:
        ms64, A64, B64, _ = run(opts64, K)
        result["fp64_path"] = {"value": 4 * K / (ms64 / 1e3), "ms_per_step": ms64 / K}
        result["speedup_vs_fp64_path"] = result["value"] / result["fp64_path"]["value"]
        # metric error of the split path on the state reached: same isometries, both precisions
        Q, Rm = ntu.ntu_reduce_qr(ctx, Am, gf[:, 0, 0].contiguous(), 0)
        QY, _ = ntu.ntu_reduce_qr(ctx, Bm, gf[:, 0, 1].contiguous(), 1)
        nb = [Bm, Bm, Bm, Am, Am, Am]
        g64 = ntu.ntu_env_contract(ctx, Q, QY, nb, "f64", D=D)
        gmx = ntu.ntu_env_contract(ctx, Q, QY, nb, args.precision, D=D)
        result["metric_rel_err_vs_fp64_path"] = float(torch.linalg.norm(gmx - g64) / torch.linalg.norm(g64))
        result["state_rel_diff_vs_fp64_path"] = float(
            torch.linalg.norm(torch.cat([Am.flatten(), Bm.flatten()]) - torch.cat([A64.flatten(), B64.flatten()]))
            / torch.linalg.norm(torch.cat([A64.flatten(), B64.flatten()])))

    # live per-kernel timing with HIP events on the library's stream
    ntu.ntu_profile_enable(ctx, True)
    run(opts, args.profile_steps)
    prof = ntu.ntu_profile_read(ctx)
    ntu.ntu_profile_enable(ctx, False)
    nprof = max(1, args.profile_steps)
    result["kernel_ms_per_step"] = {k: v[0] / nprof for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}
    R = 2 * D
    dom = max(prof.items(), key=lambda kv: kv[1][0])[0] if prof else None
    roof = {}
    if dom == "bond_fit":
        t = prof["bond_fit"][0] / prof["bond_fit"][1] / 1e3
        hs = 2 * float(iters.mean())
        fl_launch = fit_flops_per_launch(R, float(dn.mean()), hs, cplx=False)
        roof = {"kernel": "k_bond_fit", "bound": "alu", "achieved": fl_launch / t / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": fl_launch / t / PEAK_FP64, "traffic": None,
                "avg_launch_us": t * 1e6, "flops_per_launch": fl_launch}
    if "env_e6" in prof:
        t6 = prof["env_e6"][0] / prof["env_e6"][1] / 1e3
        f6 = e6_flops(R, D, cplx=False)
        e6 = {"kernel": "k_mfma_nt (metric assembly)", "bound": "mfma", "achieved": f6 / t6 / 1e12,
              "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s", "frac": f6 / t6 / PEAK_BF16, "traffic": None,
              "avg_launch_us": t6 * 1e6, "flops_per_launch": f6, "issued_mfma_flops_per_launch": 3 * f6}
        result["roofline_env_assembly"] = e6
        if not roof:
            roof = e6
    result["roofline"] = roof

    if not args.no_cpu:
        from oracle import ntu as O
        An = A0.cpu().numpy()[0]
        Bn = B0.cpu().numpy()[0]
        GAo, GBo, _ = O.gate_split(w["gates"][0], 2, 2)
        pairs = {b: (GAo, GBo) for b in O.BONDS}
        t0 = time.perf_counter()
        n_bonds = 0
        while n_bonds < 16 and time.perf_counter() - t0 < args.cpu_seconds:
            for b in O.BONDS:
                An, Bn, _ = O.trotter_step(An, Bn, pairs, D, n_iter=20, conv_tol=1e-12, order=(b,))
                n_bonds += 1
        el = time.perf_counter() - t0
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        result["cpu_baseline"] = {"value": n_bonds / el, "unit": "bond_updates/s", "cores": cores, "kind": "oracle",
                                  "sample": f"{n_bonds} bond updates of the same D=8 state (oracle FP64, numpy/BLAS)"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
