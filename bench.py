"""Throughput of one CCSD-form iteration (residual + energy + norms + Jacobi/DIIS update) on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--vvvv full|packed]
                [--generator literal|converging] [--no-cpu-baseline]

A step is one pass of the whole iteration on the device: T1 dressing, every residual term,
the energy and residual-norm reductions, the Jacobi update and DIIS (ascc_residual followed
by ascc_update), starting from T = 0 and continuing the real iteration sequence.  Inputs are
generated on the host from the seeded recipe in gen/synth_df.py and copied to HBM before the
timed region; the integral set (including the vvvv block) is built before it as well.

value = F_N6 / seconds-per-step in TFLOP/s, with the fixed algorithmic count
F_N6(o,v) = 2[T(o)T(v)^2 + S(o)S(v)^2] + 4 o^4 v^2 + 10 o^3 v^3 (T(n) = n(n+1)/2, S(n) = n(n-1)/2).

roofline: the particle-particle ladder contraction (phase pp_ladder), timed with HIP events on
the stream it runs on during the timed region; achieved = its algorithmic flops per residual
(2[T(o)T(v)^2 + S(o)S(v)^2]) / its mean duration, against the FP64 matrix peak.

cpu_baseline: the FP64 oracle (oracle/cs_ccsd.py, numpy) timed on the host for one residual
evaluation of the same workload (rank 0 only), as F_N6 / seconds.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from gen.synth_df import WORKLOADS, converging_sigma, make_system  # noqa: E402

METRIC = "N^6 residual TFLOP/s, mixed vs FP64 @|dE|<1e-6 Eh; solves/s + p99 latency"
FP64_MFMA_PEAK_TFLOPS = 78.6


def tri(n):
    return n * (n + 1) // 2


def stri(n):
    return n * (n - 1) // 2


def f_n6(o, v):
    return 2 * (tri(o) * tri(v) ** 2 + stri(o) * stri(v) ** 2) + 4 * o ** 4 * v ** 2 + 10 * o ** 3 * v ** 3


def ladder_flops(o, v):
    return 2 * (tri(o) * tri(v) ** 2 + stri(o) * stri(v) ** 2)


def cpu_baseline(B, eps, o, v):
    """One oracle residual evaluation on the host cores (bounded: a single residual)."""
    from oracle import cs_ccsd

    try:
        from threadpoolctl import threadpool_info

        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(1234)
    t1 = rng.normal(0, 0.01, (o, v))
    x = rng.normal(0, 0.01, (o, o, v, v))
    t2 = 0.5 * (x + x.transpose(1, 0, 3, 2))
    fock = np.diag(eps)
    t0 = time.perf_counter()
    cs_ccsd.residual(B, fock, t1, t2)
    cs_ccsd.energy(B, fock, t1, t2)
    dt = time.perf_counter() - t0
    return {"value": f_n6(o, v) / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one residual + energy evaluation of the same workload ({dt:.1f} s, numpy FP64)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="o20v180q600", choices=sorted(WORKLOADS))
    ap.add_argument("--vvvv", default="full", choices=["full", "packed"])
    ap.add_argument("--generator", default="literal", choices=["literal", "converging"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2501_10515_amd as P

    wl = WORKLOADS[args.workload]
    o, v, Q, seed = wl["no"], wl["nv"], wl["naux"], wl["seed"]
    sigma = converging_sigma(v, Q) if args.generator == "converging" else 0.05
    B, eps = make_system(o, v, Q, seed, sigma=sigma)
    dev = torch.device("cuda:0")
    dB = torch.from_numpy(B).to(dev)
    deps = torch.from_numpy(eps).to(dev)
    mode = P.ASCC_VVVV_FULL if args.vvvv == "full" else P.ASCC_VVVV_PACKED
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ints = P.ascc_build_ints(dB, deps, o, vvvv_mode=mode)
    build_s = time.perf_counter() - t0
    del dB

    t1 = torch.zeros((o, v), dtype=torch.float64, device=dev)
    t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device=dev)
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    stats = torch.empty(8, dtype=torch.float64, device=dev)
    diis = P.ascc_diis_create(ints, 8, 1)
    stream = torch.cuda.current_stream()

    def step():
        P.ascc_residual(ints, t1, t2, r1, r2, e)
        P.ascc_update(ints, diis, t1, t2, r1, r2, e, stats)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    P.ascc_timing_read(ints)  # discard
    P.ascc_timing_enable(ints, True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    P.ascc_timing_enable(ints, False)
    phases = P.ascc_timing_read(ints)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    flops = f_n6(o, v)
    value = flops / (ms_step * 1e-3) / 1e12

    lad_ms, lad_n = phases["pp_ladder"]
    lad_avg = lad_ms / max(lad_n, 1)
    achieved = ladder_flops(o, v) / (lad_avg * 1e-3) / 1e12
    st = stats.cpu().numpy()

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "no": o, "nv": v, "naux": Q, "seed": seed, "generator": args.generator,
            "sigma": sigma, "vvvv": args.vvvv, "precision": "fp64",
            "step": "ascc_residual + ascc_update (one Jacobi/DIIS iteration)", "flops_per_step_F_N6": flops,
        },
        "roofline": {
            "bound": "mfma", "kernel": "pp_ladder (gemm_f64_kernel)", "achieved": round(achieved, 3),
            "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
            "traffic": None, "launch_ms": round(lad_avg, 4), "algorithmic_flops_per_launch": ladder_flops(o, v),
        },
        "phases_ms_per_step": {k: round(ms / max(args.steps, 1), 4) for k, (ms, n) in phases.items() if n},
        "build_ints_s": round(build_s, 3),
        "wall_s": round(wall, 3),
        "last_stats": {"E": float(st[0]), "rnorm": float(st[3]), "finite": bool(np.isfinite(st[3]))},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(B, eps, o, v)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
