"""Throughput of one CCSD-form iteration (residual + energy + norms + Jacobi/DIIS update) on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--vvvv full|packed]
                [--precision fp64|fp32|bf16x3] [--generator literal|converging] [--no-compare]
                [--no-cpu-baseline] [--serve ...] [--solve [--ascc H,P|homo-lumo] [--plascc] [--solve-tol T]
                [--lowp-rnorm R]] [--two-ansatz ALPHA [--ascc H,P]]

A step is one pass of the whole iteration on the device: T1 dressing, every residual term,
the energy and residual-norm reductions, the Jacobi update and DIIS (ascc_residual followed
by ascc_update), starting from T = 0 and continuing the real iteration sequence.  Inputs are
generated on the host from the seeded recipe in gen/synth_df.py (by default at the
convergence-variant width, so the timed steps are a converging iteration with finite values; the
work per step does not depend on the values) and copied to HBM before the timed region; the integral set (including the vvvv block) is built before it as well.

value = F_N6 / seconds-per-step in TFLOP/s, with the fixed algorithmic count
F_N6(o,v) = 2[T(o)T(v)^2 + S(o)S(v)^2] + 4 o^4 v^2 + 10 o^3 v^3 (T(n) = n(n+1)/2, S(n) = n(n-1)/2).

roofline: the particle-particle ladder contraction (phase pp_ladder: exactly one kernel launch),
timed with HIP events on the stream it runs on during the timed region; achieved = its algorithmic
flops per launch (2[T(o)T(v)^2 + S(o)S(v)^2] per state) / its mean duration, against the matrix
peak of the arithmetic that carries it (FP64 78.6, FP32 157.3, split-BF16x3 2516.6/3 TFLOP/s);
traffic = HBM bytes per launch from rocprofv3 counters (table below), null where not measured.

variants (FP64 runs): the same workload and step with the other vvvv storage and with the N^6
contractions in FP32 and in split-BF16x3 (fewer steps each), as TFLOP/s on the same F_N6 count
and speedup over the main run; and the same step with the PLASCC term removal (primaries
HOMO -> LUMO) in FP64 and split-BF16x3, with the time of the removal itself.

cpu_baseline: the FP64 oracle (oracle/cs_ccsd.py, numpy) timed on the host for residual
evaluations of the same workload, repeated to about 10 s (rank 0 only), as F_N6 / seconds each.
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

from gen.synth_df import WORKLOADS, converging_sigma, make_system, single_excitation_guesses  # noqa: E402

METRIC = "N^6 residual TFLOP/s, mixed vs FP64 @|dE|<1e-6 Eh; solves/s + p99 latency"
FP64_MFMA_PEAK_TFLOPS = 78.6
# dense matrix peaks (TFLOP/s) of the arithmetic carrying each mode's contractions: FP64 and FP32
# MFMA; split-BF16x3 spends three BF16 products (2516.6 TFLOP/s dense) per FP32-equivalent flop
PEAKS = {"fp64": FP64_MFMA_PEAK_TFLOPS, "fp32": 157.3, "bf16x3": 2516.6 / 3}
LADDER_KERNEL = {"fp64": "gemm_f64_dma_kernel (direct-to-LDS; gemm_f64_kernel for odd strides)",
                 "fp32": "gemm_lowp_kernel",
                 "bf16x3": "gemm_bf16x3_dma_kernel or gemm_bf16x3_kernel by size"}
LADDER_SOURCE = {"fp64": "gemm_f64.hip", "fp32": "gemm_lowp.hip", "bf16x3": "gemm_lowp.hip"}

# HBM bytes per ladder launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs of this bench command,
# each scaled by what the counter reads for a plain 2 GiB copy (fetch x2.000, write x1.000), keyed by
# (workload, vvvv, precision) with the sha256 of the kernel source they were taken on: a kernel
# changed since then reports null.
TRAFFIC = {
    ("o20v180q600", "full", "fp64"): (5.331e+09, "bfd87cf674c6e0f608d28deace5a98fe722725c4e019e199fe397075f7161181"),
    ("o40v360q1200", "packed", "bf16x3"): (1.474e+11, "8692cddb0d74f53367dadd64809cd11efe62b3b5e809dd59b323e9d8e9a3f3f4"),
}


def traffic_bytes(workload, vvvv, precision):
    import hashlib

    hit = TRAFFIC.get((workload, vvvv, precision))
    if hit is None:
        return None
    src = os.path.join(ROOT, "paper_2501_10515_amd", "csrc", LADDER_SOURCE[precision])
    try:
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    return hit[0] if digest == hit[1] else None


def tri(n):
    return n * (n + 1) // 2


def stri(n):
    return n * (n - 1) // 2


def f_n6(o, v):
    return 2 * (tri(o) * tri(v) ** 2 + stri(o) * stri(v) ** 2) + 4 * o ** 4 * v ** 2 + 10 * o ** 3 * v ** 3


def ladder_flops(o, v):
    return 2 * (tri(o) * tri(v) ** 2 + stri(o) * stri(v) ** 2)


def cpu_baseline(B, eps, o, v, nstates=1):
    """Oracle residual + energy evaluations on the host cores, repeated until about 10 s of work
    (at least one, at most six), as the rate of one evaluation.

    For several states sharing the integrals the rate is that of one state's residual (the
    oracle has no batched form), which is what nstates independent evaluations would reach.
    """
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
    n = 0
    while n == 0 or (time.perf_counter() - t0 < 10.0 and n < 6):
        cs_ccsd.residual(B, fock, t1, t2)
        cs_ccsd.energy(B, fock, t1, t2)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n * f_n6(o, v) / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"{n} residual + energy evaluations of the same workload ({dt:.1f} s, numpy FP64)"
                       + (f"; each for one of its {nstates} states" if nstates > 1 else ""))}


def run_throughput(P, torch, B, eps, o, v, Q, vvvv, precision, steps, warmup, guesses=None, plascc=None):
    """Time `steps` iterations (residual + update) after `warmup` untimed ones.

    guesses None: one state from T = 0.  Otherwise one state per (i, a) pair, T2 = 0 and
    t1[i, a] = 0.5, all sharing the integral set: one ascc_residual_batch call (one ladder
    launch over every state) and one ascc_update per state, each with its own DIIS history.
    plascc (hole, particle): the same iteration with the PLASCC term removal of those primaries.
    """
    dev = torch.device("cuda:0")
    mode = P.ASCC_VVVV_FULL if vvvv == "full" else P.ASCC_VVVV_PACKED
    prec = {"fp64": P.ASCC_PREC_FP64, "fp32": P.ASCC_PREC_FP32, "bf16x3": P.ASCC_PREC_BF16X3}[precision]
    dB = torch.from_numpy(B).to(dev)
    deps = torch.from_numpy(eps).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ints = P.ascc_build_ints(dB, deps, o, precision=prec, vvvv_mode=mode)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    del dB
    if plascc is not None:
        P.ascc_set_plascc(ints, *plascc)
    nst = 1 if guesses is None else len(guesses)
    t1s = [torch.zeros((o, v), dtype=torch.float64, device=dev) for _ in range(nst)]
    t2s = [torch.zeros((o, o, v, v), dtype=torch.float64, device=dev) for _ in range(nst)]
    for k, (i, a) in enumerate(guesses or []):
        t1s[k][i, a] = 0.5
    r1s, r2s = [torch.empty_like(t) for t in t1s], [torch.empty_like(t) for t in t2s]
    e = torch.empty(nst, dtype=torch.float64, device=dev)
    stats = torch.empty((nst, 8), dtype=torch.float64, device=dev)
    diis = [P.ascc_diis_create(ints, 8, 1) for _ in range(nst)]
    stream = torch.cuda.current_stream()
    if guesses is not None:
        P.ascc_batch_reserve(ints, nst)

    def step():
        if guesses is None:
            P.ascc_residual(ints, t1s[0], t2s[0], r1s[0], r2s[0], e)
        else:
            P.ascc_residual_batch(ints, t1s, t2s, r1s, r2s, e)
        for k in range(nst):
            P.ascc_update(ints, diis[k], t1s[k], t2s[k], r1s[k], r2s[k], e[k:k + 1], stats[k])

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    P.ascc_timing_read(ints)  # discard
    P.ascc_timing_enable(ints, True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    P.ascc_timing_enable(ints, False)
    phases = P.ascc_timing_read(ints)
    ms_step = ev0.elapsed_time(ev1) / steps
    st = stats.cpu().numpy()
    for d in diis:
        d.close()
    ints.close()
    del t1s, t2s, r1s, r2s
    torch.cuda.empty_cache()
    return dict(ms_step=ms_step, wall=wall, build_s=build_s, phases=phases, steps=steps, nstates=nst,
                last={"E": [float(x) for x in st[:, 0]] if nst > 1 else float(st[0, 0]),
                      "rnorm": [float(x) for x in st[:, 3]] if nst > 1 else float(st[0, 3]),
                      "finite": bool(np.isfinite(st[:, 3]).all())})


def serve_requests(nreq: int):
    """The request stream: Poisson arrivals (mean 20/s), no ~ U{4..24}, nv = 9 no, naux = 3(no+nv).

    Arrival gaps come from default_rng(99).exponential(0.05); request k draws no and then its
    inputs (convergence-variant width) from default_rng(100 + k).
    """
    import concurrent.futures as cf

    gaps = np.random.default_rng(99).exponential(0.05, nreq)
    arrivals = np.cumsum(gaps)

    def one(k):
        rng = np.random.default_rng(100 + k)
        o = int(rng.integers(4, 25))
        v, Q = 9 * o, 3 * (10 * o)
        B, eps = make_system(o, v, Q, None, sigma=converging_sigma(v, Q), rng=rng)
        return o, B, eps

    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        reqs = list(ex.map(one, range(nreq)))
    return arrivals, reqs


def run_serving(P, arrivals, reqs, precision: int, budget: int, max_active: int, tol_rnorm: float,
                lowp_rnorm: float = 1e-5, states=()):
    srv = P.Server(budget, max_active=max_active, precision=precision, vvvv_mode=P.ASCC_VVVV_PACKED,
                   use_graphs=True, tol_rnorm=tol_rnorm, maxiter=150, lowp_rnorm=lowp_rnorm)
    n = len(reqs)
    ids = []
    t0 = time.perf_counter()
    nxt = 0
    last_print = 0.0
    while True:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            o, B, eps = reqs[nxt]
            if nxt in states:  # the HOMO -> LUMO ASCC state of this request's system
                ids.append(srv.submit(B, eps, o, float(arrivals[nxt]), hole=o - 1, particle=o))
            else:
                ids.append(srv.submit(B, eps, o, float(arrivals[nxt])))
            nxt += 1
        q, r, d = srv.step(now)
        if now - last_print > 15.0:
            print(f"serve: t={now:.1f}s submitted={nxt} queued={q} running={r} done={d}", file=sys.stderr, flush=True)
            last_print = now
        if nxt == n and d == n:
            break
        if now > 1800:
            raise TimeoutError("serving did not finish in 30 min")
        if r == 0 and nxt < n:
            time.sleep(max(0.0, min(0.002, arrivals[nxt] - now)))
    infos = [srv.info(i) for i in ids]
    srv.close()
    lat = np.array([x["t_done"] - x["t_submit"] for x in infos])
    done = max(x["t_done"] for x in infos)
    ok = sum(1 for x in infos if x["status"] == 0)
    st = [x for x in infos if x["hole"] >= 0]
    extra = {}
    if st:
        lst = np.array([x["t_done"] - x["t_submit"] for x in st])
        extra = dict(states=len(st), states_converged=sum(1 for x in st if x["status"] == 0),
                     states_p50_s=float(np.percentile(lst, 50)), states_p99_s=float(np.percentile(lst, 99)),
                     states_mean_iterations=float(np.mean([x["iterations"] for x in st])))
    return dict(solves_per_s=n / (done - float(arrivals[0])), p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), converged=ok, n=n, **extra,
                mean_iterations=float(np.mean([x["iterations"] for x in infos])),
                mean_lowp_iterations=float(np.mean([x["lowp_iterations"] for x in infos])),
                energies=[x["e_corr"] for x in infos])


def serve_main(args):
    import torch  # noqa: F401

    import paper_2501_10515_amd as P

    arrivals, reqs = serve_requests(args.requests)
    # --serve-states F: every request k with k % round(1/F) == 0 asks for its HOMO -> LUMO ASCC state
    states = set(range(0, args.requests, max(1, round(1.0 / args.serve_states)))) if args.serve_states > 0 else set()
    budget = int(args.budget_gb * (1 << 30))
    out = {"metric": "served solves/s (continuous batching, Poisson arrivals 20 req/s)", "unit": "solves/s",
           "n_gpus": 1, "data": "synthetic", "dtype": "f64",
           "config": {"workload": f"serve{args.requests}", "arrival_rate_per_s": 20, "no": "U{4..24}",
                      "nv": "9 no", "naux": "3 (no + nv)", "seeds": f"100..{99 + args.requests}",
                      "generator": "converging", "hbm_budget_gb": args.budget_gb, "max_active": args.max_active,
                      "tol_rnorm": args.serve_tol, "lowp_rnorm": args.lowp_rnorm, "vvvv": "packed",
                      "excited_state_requests": len(states)}}
    res = {}
    for name, pc in (("bf16x3_refined", P.ASCC_PREC_BF16X3), ("fp32_refined", P.ASCC_PREC_FP32),
                     ("fp64", P.ASCC_PREC_FP64)):
        if args.serve_precisions and name.split("_")[0] not in args.serve_precisions.split(","):
            continue
        r = run_serving(P, arrivals, reqs, pc, budget, args.max_active, args.serve_tol, args.lowp_rnorm, states)
        res[name] = r
        print(f"serving mode {name}: {r['solves_per_s']:.3f} solves/s", file=sys.stderr, flush=True)
    base = res.get("fp64")
    for name, r in res.items():
        if base is not None and name != "fp64":
            r["max_abs_dE_vs_fp64"] = float(max(abs(a - b) for a, b in zip(r["energies"], base["energies"])))
    for r in res.values():
        r.pop("energies")
    main = res.get("bf16x3_refined") or next(iter(res.values()))
    out["value"] = round(main["solves_per_s"], 4)
    out["higher_is_better"] = True
    out["vs_baseline"] = None
    out["p50_s"] = round(main["p50_s"], 4)
    out["p99_s"] = round(main["p99_s"], 4)
    out["modes"] = res
    print(json.dumps(out), flush=True)


def criterion(args) -> dict:
    """Convergence test of the solves: |R|_2 <= --solve-tol, or with --paper-criterion the paper's own
    (Sec. III.A): max|R| <= 1e-5 and |dE| < 1e-7 Eh in one iteration."""
    if args.paper_criterion:
        return dict(tol_rnorm=0.0, tol_rmax=1e-5, tol_de=1e-7)
    return dict(tol_rnorm=args.solve_tol)


def solve_main(args):
    """Precision study: one workload (convergence-variant generator) solved to the same tolerance with
    FP64 contractions and with low-precision bulk iterations finished in FP64; |dE| against FP64."""
    import torch

    import paper_2501_10515_amd as P

    wl = WORKLOADS[args.workload]
    o, v, Q, seed = wl["no"], wl["nv"], wl["naux"], wl["seed"]
    sigma = converging_sigma(v, Q)
    B, eps = make_system(o, v, Q, seed, sigma=sigma)
    dev = torch.device("cuda:0")
    state = None  # (hole, particle) of an ASCC 1-CSF state, else the ground state
    if args.ascc:
        hole, particle = (int(x) for x in args.ascc.split(",")) if args.ascc != "homo-lumo" else (o - 1, o)
        state = (hole, particle)

    prim = None  # primaries of the PLASCC term removal
    if args.plascc:
        prim = state if state is not None else (o - 1, o)

    def build(dB, deps, pc, mode):
        if state is None:
            ints = P.ascc_build_ints(dB, deps, o, precision=pc, vvvv_mode=mode)
        else:
            ints = P.ascc_build_ints_hbar(dB, deps, o, state[0], state[1], precision=pc, vvvv_mode=mode)
        if prim is not None:
            P.ascc_set_plascc(ints, *prim)
        return ints

    def start(t1, t2):  # T = 0, or the ASCC guess T^P(0) = S - S^2/2
        if state is None:
            t1.zero_()
            t2.zero_()
        else:
            P.ascc_initial_guess(t1, t2, state[0], state[1])
    mode = P.ASCC_VVVV_FULL if args.vvvv == "full" else P.ASCC_VVVV_PACKED
    crit = criterion(args)
    res = {}
    for name, pc, lowp_rnorm in (("fp64", P.ASCC_PREC_FP64, 0.0), ("bf16x3_refined", P.ASCC_PREC_BF16X3, args.lowp_rnorm),
                                 ("fp32_refined", P.ASCC_PREC_FP32, args.lowp_rnorm)):
        if args.serve_precisions and name.split("_")[0] not in args.serve_precisions.split(","):
            continue
        dB, deps = torch.from_numpy(B).to(dev), torch.from_numpy(eps).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ints = build(dB, deps, pc, mode)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        del dB
        t1 = torch.zeros((o, v), dtype=torch.float64, device=dev)
        t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device=dev)
        # untimed one-iteration solve first: the solver's DIIS history and work arrays (tens of GB
        # here) are then no longer the first touch of fresh device memory inside the timed solve
        start(t1, t2)
        P.ascc_solve(ints, t1, t2, maxiter=1, lowp_rnorm=lowp_rnorm, raise_on_not_converged=False, **crit)
        start(t1, t2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = P.ascc_solve(ints, t1, t2, maxiter=args.solve_maxiter, lowp_rnorm=lowp_rnorm,
                         raise_on_not_converged=False, **crit)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        print(f"solve mode {name}: {t_solve:.2f} s, {r['iterations']} iterations", file=sys.stderr, flush=True)
        res[name] = {"e_corr": r["e_corr"], "rnorm": r["rnorm"], "rmax": r["rmax"], "iterations": r["iterations"],
                     "lowp_iterations": r["lowp_iterations"], "converged": r["converged"],
                     "solve_s": round(t_solve, 3), "build_s": round(t_build, 3),
                     "e_total": P.ascc_reference_energy(ints) + r["e_corr"]}
        ints.close()
        del t1, t2
        torch.cuda.empty_cache()
    base = res.get("fp64")
    for name, r in res.items():
        if base is not None and name != "fp64":
            r["abs_dE_vs_fp64"] = abs(r["e_corr"] - base["e_corr"])
            r["speedup_vs_fp64"] = round(base["solve_s"] / r["solve_s"], 3)
    ground = None
    if state is not None:  # the ground state of the same system, FP64: the excitation energy
        dB, deps = torch.from_numpy(B).to(dev), torch.from_numpy(eps).to(dev)
        ints = P.ascc_build_ints(dB, deps, o, vvvv_mode=mode)
        if prim is not None:  # the same removal in the ground state (Sec. II.C)
            P.ascc_set_plascc(ints, *prim)
        del dB
        t1 = torch.zeros((o, v), dtype=torch.float64, device=dev)
        t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device=dev)
        r = P.ascc_solve(ints, t1, t2, maxiter=args.solve_maxiter, raise_on_not_converged=False, **crit)
        ground = {"e_total": P.ascc_reference_energy(ints) + r["e_corr"], "iterations": r["iterations"],
                  "converged": r["converged"]}
        ints.close()
        del t1, t2
        torch.cuda.empty_cache()
        for rr in res.values():
            rr["excitation_energy_eV"] = round((rr["e_total"] - ground["e_total"]) * 27.211386, 6)
    main = res.get("bf16x3_refined") or next(iter(res.values()))
    what = "ground state" if state is None else f"ASCC 1-CSF state {state[0]}->{state[1]} (transformed Hamiltonian)"
    if prim is not None:
        what = f"PLASCC ({prim[0]}->{prim[1]} primaries), " + what
    out = {"metric": f"time to converged energy, mixed vs FP64 (|dE| < 1e-6 Eh), {what}", "unit": "s",
           "value": main["solve_s"], "higher_is_better": False, "n_gpus": 1, "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": args.workload, "no": o, "nv": v, "naux": Q, "seed": seed, "generator": "converging",
                      "sigma": sigma, "vvvv": args.vvvv, "criterion": crit, "lowp_rnorm": args.lowp_rnorm,
                      "state": "ground" if state is None else {"hole": state[0], "particle": state[1],
                                                                "guess": "T^P(0) = S - S^2/2"},
                      "plascc_primaries": list(prim) if prim is not None else None},
           "modes": res}
    if ground is not None:
        out["ground_state_fp64"] = ground
    print(json.dumps(out), flush=True)


def two_ansatz_main(args):
    """Both ansatz of a 1-CSF state (Aufbau coefficient --two-ansatz ALPHA) per precision mode: the
    time of the pair of solves (each integral set built, solved and freed in turn), both total
    energies and their mean."""
    import torch

    import paper_2501_10515_amd as P

    wl = WORKLOADS[args.workload]
    o, v, Q, seed = wl["no"], wl["nv"], wl["naux"], wl["seed"]
    sigma = converging_sigma(v, Q)
    B, eps = make_system(o, v, Q, seed, sigma=sigma)
    dev = torch.device("cuda:0")
    hole, particle = (int(x) for x in args.ascc.split(",")) if args.ascc not in ("", "homo-lumo") else (o - 1, o)
    mode = P.ASCC_VVVV_FULL if args.vvvv == "full" else P.ASCC_VVVV_PACKED
    dB, deps = torch.from_numpy(B).to(dev), torch.from_numpy(eps).to(dev)
    t1s = [torch.empty((o, v), dtype=torch.float64, device=dev) for _ in range(2)]
    t2s = [torch.empty((o, o, v, v), dtype=torch.float64, device=dev) for _ in range(2)]
    res = {}
    for name, pc, lowp in (("fp64", P.ASCC_PREC_FP64, 0.0), ("bf16x3_refined", P.ASCC_PREC_BF16X3, args.lowp_rnorm)):
        if args.serve_precisions and name.split("_")[0] not in args.serve_precisions.split(","):
            continue
        kw = dict(precision=pc, vvvv_mode=mode, lowp_rnorm=lowp, raise_on_not_converged=False, **criterion(args))
        P.ascc_two_ansatz(dB, deps, o, hole, particle, args.two_ansatz, t1s, t2s, maxiter=1, **kw)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = P.ascc_two_ansatz(dB, deps, o, hole, particle, args.two_ansatz, t1s, t2s, maxiter=args.solve_maxiter, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"two-ansatz mode {name}: {dt:.2f} s", file=sys.stderr, flush=True)
        res[name] = {"seconds": round(dt, 3), "e_total": r["e_total"], "e_mean": r["e_mean"], "beta": r["beta"],
                     "solves": r["solves"]}
    base = res.get("fp64")
    for name, r in res.items():
        if base is not None and name != "fp64":
            r["abs_dE_mean_vs_fp64"] = abs(r["e_mean"] - base["e_mean"])
            r["speedup_vs_fp64"] = round(base["seconds"] / r["seconds"], 3)
    main = res.get("bf16x3_refined") or next(iter(res.values()))
    out = {"metric": "time to the two-ansatz ASCC energy (both solves), mixed vs FP64", "unit": "s",
           "value": main["seconds"], "higher_is_better": False, "n_gpus": 1, "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": args.workload, "no": o, "nv": v, "naux": Q, "seed": seed, "generator": "converging",
                      "sigma": sigma, "vvvv": args.vvvv, "criterion": criterion(args), "lowp_rnorm": args.lowp_rnorm,
                      "hole": hole, "particle": particle, "alpha": args.two_ansatz},
           "modes": res}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="o20v180q600", choices=sorted(WORKLOADS))
    ap.add_argument("--vvvv", default="full", choices=["full", "packed"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--generator", default="converging", choices=["literal", "converging"],
                    help="integral width: the convergence variant (default) or the literal sigma = 0.05")
    ap.add_argument("--no-compare", action="store_true", help="skip the low-precision comparison runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true", help="run the request-serving workload instead")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-active", type=int, default=32)
    ap.add_argument("--serve-tol", type=float, default=1e-7)
    ap.add_argument("--serve-precisions", default="", help="comma list of fp64,fp32,bf16x3 (default all)")
    ap.add_argument("--serve-states", type=float, default=0.0,
                    help="fraction of requests that ask for an ASCC excited state (HOMO -> LUMO) instead")
    ap.add_argument("--solve", action="store_true", help="precision study: full solves of --workload per mode")
    ap.add_argument("--ascc", default="", help="with --solve: an ASCC 1-CSF state, 'hole,particle' (orbital "
                    "indices) or 'homo-lumo', solved on its transformed Hamiltonian from T^P(0)")
    ap.add_argument("--plascc", action="store_true", help="with --solve: the PLASCC term removal, primaries of "
                    "--ascc (or HOMO -> LUMO for the ground state), in every solve")
    ap.add_argument("--two-ansatz", type=float, default=None, metavar="ALPHA",
                    help="both ansatz of the --ascc state (default HOMO -> LUMO) for Aufbau coefficient ALPHA")
    ap.add_argument("--solve-tol", type=float, default=1e-7)
    ap.add_argument("--paper-criterion", action="store_true",
                    help="solves converge on max|R| <= 1e-5 and |dE| < 1e-7 Eh instead of --solve-tol")
    ap.add_argument("--solve-maxiter", type=int, default=60)
    ap.add_argument("--lowp-rnorm", type=float, default=1e-7,
                    help="hand-over residual norm of the low-precision bulk (the rounding-floor test also applies)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve_main(args)
        return
    if args.two_ansatz is not None:
        two_ansatz_main(args)
        return
    if args.solve:
        solve_main(args)
        return

    import torch

    import paper_2501_10515_amd as P

    wl = WORKLOADS[args.workload]
    o, v, Q, seed = wl["no"], wl["nv"], wl["naux"], wl["seed"]
    sigma = converging_sigma(v, Q) if args.generator == "converging" else 0.05
    rng = np.random.default_rng(seed)
    B, eps = make_system(o, v, Q, seed, sigma=sigma, rng=rng)
    nstates = wl.get("nstates", 1)
    guesses = single_excitation_guesses(o, v, nstates, rng) if nstates > 1 else None
    flops = nstates * f_n6(o, v)

    main_run = run_throughput(P, torch, B, eps, o, v, Q, args.vvvv, args.precision, args.steps, args.warmup,
                              guesses)
    ms_step = main_run["ms_step"]
    value = flops / (ms_step * 1e-3) / 1e12
    phases = main_run["phases"]
    lad_ms, lad_n = phases["pp_ladder"]
    lad_avg = lad_ms / max(lad_n, 1)
    achieved = nstates * ladder_flops(o, v) / (lad_avg * 1e-3) / 1e12
    peak = PEAKS[args.precision]

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
            "workload": args.workload, "no": o, "nv": v, "naux": Q, "seed": seed, "nstates": nstates,
            "generator": args.generator,
            "sigma": sigma, "vvvv": args.vvvv, "precision": args.precision,
            "step": ("ascc_residual + ascc_update (one Jacobi/DIIS iteration)" if nstates == 1 else
                     f"ascc_residual_batch over {nstates} states + {nstates} x ascc_update"),
            "flops_per_step_F_N6": flops,
        },
        "roofline": {
            "bound": "mfma", "kernel": f"pp_ladder ({LADDER_KERNEL[args.precision]}, one launch)",
            "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": traffic_bytes(args.workload, args.vvvv, args.precision), "launch_ms": round(lad_avg, 4),
            "algorithmic_flops_per_launch": nstates * ladder_flops(o, v),
        },
        "phases_ms_per_step": {k: round(ms / main_run["steps"], 4) for k, (ms, n) in phases.items() if n},
        "build_ints_s": round(main_run["build_s"], 3),
        "wall_s": round(main_run["wall"], 3),
        "last_stats": main_run["last"],
    }
    if not args.no_compare and args.precision == "fp64":
        comp = {}
        other = "packed" if args.vvvv == "full" else "full"
        for vm, pr, pl in ((other, "fp64", None), (args.vvvv, "fp32", None), (args.vvvv, "bf16x3", None),
                           ("packed", "bf16x3", None), (args.vvvv, "fp64", (o - 1, o)), (args.vvvv, "bf16x3", (o - 1, o))):
            key = f"{pr}_{vm}" + ("_plascc" if pl else "")
            if key in comp or (pl and nstates > 1):
                continue
            try:
                r = run_throughput(P, torch, B, eps, o, v, Q, vm, pr, max(3, args.steps // 3), min(2, args.warmup),
                                   guesses, plascc=pl)
                rl, rn = r["phases"]["pp_ladder"]
                lms = rl / max(rn, 1)
                lach = nstates * ladder_flops(o, v) / (lms * 1e-3) / 1e12
                comp[key] = {"tflops": round(flops / (r["ms_step"] * 1e-3) / 1e12, 3),
                             "ms_per_step": round(r["ms_step"], 4),
                             "speedup_vs_main": round(ms_step / r["ms_step"], 3),
                             "pp_ladder_ms": round(lms, 4),
                             # the ladder against the peak of the arithmetic that carries it
                             "pp_ladder_tflops": round(lach, 3),
                             "pp_ladder_frac": round(lach / PEAKS[pr], 4)}
                if pl:  # the PLASCC removal (primaries HOMO -> LUMO) and its own phase
                    pms, pn = r["phases"].get("plascc", (0.0, 0))
                    comp[key]["plascc_primaries"] = list(pl)
                    comp[key]["plascc_phase_ms"] = round(pms / max(r["steps"], 1), 4)
            except Exception as exc:  # keep the primary measurement if a comparison fails
                comp[key] = {"error": str(exc)[:200]}
        out["variants"] = comp
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(B, eps, o, v, nstates)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
