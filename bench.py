"""Throughput of one CCSD-form iteration (residual + energy + norms + Jacobi/DIIS update) on one MI355X,
FP64 against the mixed-precision modes at the |dE| < 1e-6 Eh gate, plus the served-request stream.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--vvvv full|packed]
                [--generator literal|converging] [--no-compare] [--no-solves] [--no-serve]
                [--no-counters] [--no-cpu-baseline]
python bench.py --serve ... | --solve [--ascc H,P|homo-lumo] [--plascc] ... | --two-ansatz ALPHA ...

A step is one pass of the whole iteration on the device: T1 dressing, every residual term, the
energy and residual-norm reductions, the Jacobi update and DIIS (ascc_residual followed by
ascc_update), starting from T = 0 and continuing the real iteration sequence.  Inputs are generated
on the host from the seeded recipe in gen/synth_df.py (by default at the convergence-variant width,
so the timed steps are a converging iteration with finite values; the work per step does not depend
on the values) and copied to HBM before the timed region; the integral set (including the vvvv
block) is built before it as well.

Default run (workload o40 v360 Q1200, seed 2, packed vvvv -- the precision-study configuration and
the largest single-solve one):
* value: the FP64 step, as F_N6 / seconds-per-step in TFLOP/s with the fixed algorithmic count
  F_N6(o,v) = 2[T(o)T(v)^2 + S(o)S(v)^2] + 4 o^4 v^2 + 10 o^3 v^3 (T(n) = n(n+1)/2, S(n) = n(n-1)/2);
* variants: the same step with the N^6 contractions in split-BF16x3 and in FP32 (speedup over FP64),
  each with |dE_corr| and max|R| of a refined solve (low-precision bulk, FP64 finish) against the
  FP64 GPU solve of the same workload, all to |R|_2 <= 1e-7 on an FP64 residual; and the o20 v180
  Q600 FP64 step with the full (ac|bd) block materialised;
* roofline: the dominant kernel by time, the ring products (one launch of Y1 = Tx K and Y2 = U L,
  one of P1 and P2: 2 x 2 (ov)^3 flops each), timed with HIP events on the library's stream;
  traffic and MFMA utilisation from rocprofv3 counter runs of this same workload launched by this
  run (--no-counters: null), each FETCH_SIZE / WRITE_SIZE scaled by what it reads for a plain
  device copy of known size in the same run;
* serving: the 256-request Poisson stream (20 req/s), split-BF16x3 refined and FP64;
* cpu_baseline: the FP64 oracle (oracle/cs_ccsd.py, numpy) on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import tempfile
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
SIMDS = 256 * 4  # MI355X: 256 compute units of 4 SIMDs (MFMA utilisation denominator)
XCDS = 8  # GRBM_GUI_ACTIVE comes per XCD; rocprofv3's CSV row is the sum over the 8 instances
EXCITED_LABEL = "ASCC 1-CSF state, T1 + T2 (the mixed triples T^M_3' are not included)"


def tri(n):
    return n * (n + 1) // 2


def stri(n):
    return n * (n - 1) // 2


def f_n6(o, v):
    return 2 * (tri(o) * tri(v) ** 2 + stri(o) * stri(v) ** 2) + 4 * o ** 4 * v ** 2 + 10 * o ** 3 * v ** 3


def ladder_flops(o, v):
    return 2 * (tri(o) * tri(v) ** 2 + stri(o) * stri(v) ** 2)


def _host_info():
    info = {"affinity_cores": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable"):
                    info["mem_available_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


def _oracle_rate(o, v, Q, seed, budget_s, max_evals):
    """Oracle residual + energy evaluations of one workload (converging width, random amplitudes),
    repeated until about budget_s seconds of work (at least one), as F_N6 per second."""
    from oracle import cs_ccsd

    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    rng = np.random.default_rng(1234)
    t1 = rng.normal(0, 0.01, (o, v))
    x = rng.normal(0, 0.01, (o, o, v, v))
    t2 = 0.5 * (x + x.transpose(1, 0, 3, 2))
    fock = np.diag(eps)
    t0 = time.perf_counter()
    n = 0
    while n == 0 or (time.perf_counter() - t0 < budget_s and n < max_evals):
        cs_ccsd.residual(B, fock, t1, t2)
        cs_ccsd.energy(B, fock, t1, t2)
        n += 1
    dt = time.perf_counter() - t0
    return n, dt, n * f_n6(o, v) / dt


def cpu_baseline(o, v, Q, seed, nstates=1):
    """The FP64 oracle timed on the host cores (all BLAS threads), and once more on one thread.

    At o40 v360 Q1200 one oracle residual is 4.5e13 flops (several minutes of host work, and its
    plain (ac|bd) block alone is 134 GB), so the bounded sample is the oracle on the o20 v180 Q600
    workload of the same generator (v/o = 9, Q = 3n), repeated to about 10 s: a stand-in rate, said
    so in `sample`.  Smaller workloads are sampled themselves.  The single-thread rate uses o12 v108
    Q360 (one evaluation of about 3e10 flops) for the same reason.
    """
    from threadpoolctl import threadpool_info, threadpool_limits

    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    stand_in = f_n6(o, v) > 2e12
    wo, wv, wq, ws = (20, 180, 600, 1) if stand_in else (o, v, Q, seed)
    n, dt, rate = _oracle_rate(wo, wv, wq, ws, 10.0, 6)
    with threadpool_limits(limits=1):
        n1, dt1, rate1 = _oracle_rate(12, 108, 360, 5, 5.0, 3)
    sample = (f"{n} oracle residual + energy evaluations of o{wo} v{wv} Q{wq} ({dt:.1f} s, numpy FP64, "
              f"{threads} BLAS threads)")
    if stand_in:
        sample += (f"; stand-in for o{o} v{v} Q{Q}, whose single oracle residual ({f_n6(o, v):.2e} flops) is "
                   f"beyond a bounded sample")
    if nstates > 1:
        sample += f"; each for one of its {nstates} states"
    return {"value": rate / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle", "sample": sample,
            "single_thread": {"value": rate1 / 1e12, "unit": "TFLOP/s", "cores": 1,
                              "sample": f"{n1} evaluations of o12 v108 Q360 ({dt1:.1f} s)"},
            "host": _host_info()}


def build_handle(P, torch, B, eps, o, vvvv, precision):
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
    del dB, deps
    ints.bench_build = (prec, mode)
    return ints, build_s


def timed_steps(P, torch, ints, o, v, precision, steps, warmup, guesses=None, plascc=None):
    """Time `steps` iterations (residual + update) after `warmup` untimed ones, from T = 0 (or, with
    guesses, one state per (i, a) pair with t1[i, a] = 0.5 sharing the integral set: one
    ascc_residual_batch call and one ascc_update per state), in `precision` on a handle that holds it.
    plascc (hole, particle): the same iteration with the PLASCC term removal of those primaries."""
    dev = torch.device("cuda:0")
    P.ascc_set_precision(ints, {"fp64": P.ASCC_PREC_FP64, "fp32": P.ASCC_PREC_FP32,
                                "bf16x3": P.ASCC_PREC_BF16X3}[precision])
    if plascc is not None:
        P.ascc_set_plascc(ints, *plascc)
    nst = 1 if guesses is None else len(guesses)
    # the states' arrays stacked (evenly spaced), so a batch runs its terms in grouped passes
    T1 = torch.zeros((nst, o, v), dtype=torch.float64, device=dev)
    T2 = torch.zeros((nst, o, o, v, v), dtype=torch.float64, device=dev)
    for k, (i, a) in enumerate(guesses or []):
        T1[k, i, a] = 0.5
    R1, R2 = torch.empty_like(T1), torch.empty_like(T2)
    t1s, t2s, r1s, r2s = list(T1), list(T2), list(R1), list(R2)
    e = torch.empty(nst, dtype=torch.float64, device=dev)
    stats = torch.empty((nst, 8), dtype=torch.float64, device=dev)
    diis = [P.ascc_diis_create(ints, 8, 1) for _ in range(nst)]
    stream = torch.cuda.current_stream()
    group = 1
    if guesses is not None:
        # states per grouped pass: as many work-array copies (up to 4) as 80% of the free memory holds
        pc, vm = ints.bench_build  # the precision and vvvv storage the handle was built with
        base = P.ascc_batch_workspace_bytes(o, v, ints.naux, nst, 1, precision=pc, vvvv_mode=vm)
        block = P.ascc_batch_workspace_bytes(o, v, ints.naux, nst, 2, precision=pc, vvvv_mode=vm) - base
        free = torch.cuda.mem_get_info()[0]
        group = int(max(1, min(4, nst, (0.8 * free - base) // max(block, 1))))
        P.ascc_batch_reserve_ws(ints, nst, group)

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
    if plascc is not None:
        P.ascc_set_plascc(ints, -1)
    del t1s, t2s, r1s, r2s, T1, T2, R1, R2
    torch.cuda.empty_cache()
    return dict(ms_step=ms_step, wall=wall, phases=phases, steps=steps, nstates=nst, group=group,
                last={"E": [float(x) for x in st[:, 0]] if nst > 1 else float(st[0, 0]),
                      "rnorm": [float(x) for x in st[:, 3]] if nst > 1 else float(st[0, 3]),
                      "finite": bool(np.isfinite(st[:, 3]).all())})


def run_throughput(P, torch, B, eps, o, v, Q, vvvv, precision, steps, warmup, guesses=None, plascc=None):
    """timed_steps on a handle built for this precision (freed afterwards)."""
    ints, build_s = build_handle(P, torch, B, eps, o, vvvv, precision)
    r = timed_steps(P, torch, ints, o, v, precision, steps, warmup, guesses, plascc)
    ints.close()
    torch.cuda.empty_cache()
    r["build_s"] = build_s
    return r


def timed_solve(P, torch, ints, o, v, precision, tol_rnorm, maxiter=60):
    """A solve from T = 0 to |R|_2 <= tol_rnorm (low-precision bulk + FP64 finish for fp32 / bf16x3)
    after an untimed one-iteration solve (so that the solver's DIIS history is not first-touch
    device memory inside the timed solve)."""
    dev = torch.device("cuda:0")
    P.ascc_set_precision(ints, {"fp64": P.ASCC_PREC_FP64, "fp32": P.ASCC_PREC_FP32,
                                "bf16x3": P.ASCC_PREC_BF16X3}[precision])
    lowp = 0.0 if precision == "fp64" else tol_rnorm
    t1 = torch.zeros((o, v), dtype=torch.float64, device=dev)
    t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device=dev)
    P.ascc_solve(ints, t1, t2, maxiter=1, tol_rnorm=tol_rnorm, lowp_rnorm=lowp, raise_on_not_converged=False)
    t1.zero_()
    t2.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = P.ascc_solve(ints, t1, t2, maxiter=maxiter, tol_rnorm=tol_rnorm, lowp_rnorm=lowp,
                     raise_on_not_converged=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del t1, t2
    torch.cuda.empty_cache()
    return {"e_corr": r["e_corr"], "rnorm": r["rnorm"], "max_abs_R": r["rmax"], "iterations": r["iterations"],
            "lowp_iterations": r["lowp_iterations"], "converged": r["converged"], "solve_s": round(dt, 3)}


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
    # only converged requests count as solves; latency percentiles are over every request
    return dict(solves_per_s=ok / (done - float(arrivals[0])), p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), converged=ok, n=n, **extra,
                mean_iterations=float(np.mean([x["iterations"] for x in infos])),
                mean_lowp_iterations=float(np.mean([x["lowp_iterations"] for x in infos])),
                energies=[x["e_corr"] for x in infos], statuses=[x["status"] for x in infos])


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
    gate_serving(res)
    main = res.get("bf16x3_refined") or next(iter(res.values()))
    out["value"] = round(main["solves_per_s"], 4)
    out["higher_is_better"] = True
    out["vs_baseline"] = None
    out["p50_s"] = round(main["p50_s"], 4)
    out["p99_s"] = round(main["p99_s"], 4)
    out["valid"] = main["valid"]
    out["modes"] = res
    print(json.dumps(out), flush=True)


def gate_serving(res):
    """|dE| of every low-precision mode against the FP64 mode's energies, request by request, and the
    validity of each mode's rate: every request converged and (low precision) max|dE| < 1e-6 Eh."""
    base = res.get("fp64")
    for name, r in res.items():
        both = [(a, b) for a, b, sa, sb in zip(r["energies"], base["energies"], r["statuses"], base["statuses"])
                if sa == 0 and sb == 0] if base is not None and name != "fp64" else []
        if both:
            r["max_abs_dE_vs_fp64"] = float(max(abs(a - b) for a, b in both))
        r["valid"] = bool(r["converged"] == r["n"] and r.get("max_abs_dE_vs_fp64", 0.0) < 1e-6)
        if not r["valid"]:
            print(f"serving mode {name}: INVALID (converged {r['converged']}/{r['n']}, "
                  f"max|dE| {r.get('max_abs_dE_vs_fp64')})", file=sys.stderr, flush=True)
    for r in res.values():
        r.pop("energies")
        r.pop("statuses")


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
    what = "ground state" if state is None else (f"{EXCITED_LABEL}: {state[0]}->{state[1]} on its transformed "
                                                 f"Hamiltonian")
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
           "state": EXCITED_LABEL,
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
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="o40v360q1200", choices=sorted(WORKLOADS))
    ap.add_argument("--vvvv", default="packed", choices=["full", "packed"])
    ap.add_argument("--generator", default="converging", choices=["literal", "converging"],
                    help="integral width: the convergence variant (default) or the literal sigma = 0.05")
    ap.add_argument("--no-compare", action="store_true", help="skip the low-precision comparison runs")
    ap.add_argument("--no-solves", action="store_true", help="skip the precision-gate solves")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream in the default run")
    ap.add_argument("--no-counters", action="store_true", help="skip the rocprofv3 counter passes")
    ap.add_argument("--counter-child", action="store_true", help=argparse.SUPPRESS)
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
                    "--ascc (or HOMO -> LUMO for the ground state), in every solve; without --solve: an extra "
                    "FP64 step variant with the removal (HOMO -> LUMO)")
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

    if args.counter_child:
        counter_child(args)
        return
    headline(args)


def ring_flops(o, v):
    """One ring launch: two [ov x ov] . [ov x ov] products (Y1 and Y2, or P1 and P2)."""
    return 2 * 2 * (o * v) ** 3


def phase_avg(phases, name):
    ms, n = phases.get(name, (0.0, 0))
    return ms / n if n else None


def step_summary(run, flops, o, v, prec, nstates=1):
    ph = run["phases"]
    lad = phase_avg(ph, "pp_ladder")
    out = {"tflops": round(flops / (run["ms_step"] * 1e-3) / 1e12, 3), "ms_per_step": round(run["ms_step"], 4),
           "pp_ladder_ms": round(lad, 4)}
    lach = nstates * ladder_flops(o, v) / (lad * 1e-3) / 1e12
    out["pp_ladder_tflops"] = round(lach, 3)
    out["pp_ladder_frac"] = round(lach / PEAKS[prec], 4)
    ry, rp = ph.get("ring_y", (0.0, 0)), ph.get("ring_p", (0.0, 0))
    if ry[1] and rp[1]:
        # per step, each state's two ring launches (several states share a launch in a grouped
        # pass); in the low modes ring_p also holds the shadow of its operand
        ms_step_rings = (ry[0] + rp[0]) / run["steps"]
        rach = 2 * nstates * ring_flops(o, v) / (ms_step_rings * 1e-3) / 1e12
        out["ring_ms"] = round((ry[0] + rp[0]) / (ry[1] + rp[1]), 4)  # per launch
        out["ring_ms_per_step"] = round(ms_step_rings, 4)
        out["ring_tflops"] = round(rach, 3)
        out["ring_frac"] = round(rach / PEAKS[prec], 4)
    out["phases_ms_per_step"] = {k: round(ms / run["steps"], 4) for k, (ms, n) in ph.items() if n}
    return out


def headline(args):
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
    compare = not args.no_compare
    log = lambda msg: print(msg, file=sys.stderr, flush=True)  # noqa: E731

    # one integral set holding the FP64 operands and their split-BF16x3 shadows: the FP64 step, the
    # split-BF16x3 step and both solves of the precision gate run on it
    ints, build_s = build_handle(P, torch, B, eps, o, args.vvvv, "bf16x3" if compare else "fp64")
    log(f"built o{o} v{v} Q{Q} ({args.vvvv}) in {build_s:.2f} s")
    main_run = timed_steps(P, torch, ints, o, v, "fp64", args.steps, args.warmup, guesses)
    ms_step = main_run["ms_step"]
    log(f"fp64 step {ms_step:.3f} ms")
    phases = main_run["phases"]
    fp64 = step_summary(main_run, flops, o, v, "fp64", nstates)
    ring_ms = fp64.get("ring_ms")
    out = {
        "metric": METRIC,
        "value": round(flops / (ms_step * 1e-3) / 1e12, 4),
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
            "generator": args.generator, "sigma": sigma, "vvvv": args.vvvv, "precision": "fp64",
            "step": ("ascc_residual + ascc_update (one Jacobi/DIIS iteration)" if nstates == 1 else
                     f"ascc_residual_batch over {nstates} states (one pp-ladder launch for all, the other terms "
                     f"in batched passes of {main_run.get('group')} states) + {nstates} x ascc_update (FP64 "
                     f"master amplitudes per state, wider than the FP32 sets the workload names)"),
            "flops_per_step_F_N6": flops,
        },
        "roofline": {
            "bound": "mfma",
            "kernel": "ring products: gemm_f64_dma_kernel 192x192, one launch per pair (Y1 = Tx K with Y2 = U L, "
                      "then P1 with P2)",
            "achieved": fp64.get("ring_tflops"), "peak": PEAKS["fp64"], "unit": "TFLOP/s",
            "frac": fp64.get("ring_frac"), "traffic": None, "launch_ms": ring_ms,
            "algorithmic_flops_per_launch": main_run.get("group", 1) * ring_flops(o, v),
            "share_of_step": round(fp64["ring_ms_per_step"] / ms_step, 4) if ring_ms else None,
        },
        "fp64_step": fp64,
        "phases_ms_per_step": {k: round(ms / main_run["steps"], 4) for k, (ms, n) in phases.items() if n},
        "build_ints_s": round(build_s, 3),
        "wall_s": round(main_run["wall"], 3),
        "last_stats": main_run["last"],
    }
    variants, gate = {}, {}
    if args.plascc and nstates == 1:  # the same FP64 step with the PLASCC removal (HOMO -> LUMO primaries)
        r = timed_steps(P, torch, ints, o, v, "fp64", args.steps, args.warmup, guesses, plascc=(o - 1, o))
        variants["fp64_plascc"] = step_summary(r, flops, o, v, "fp64", nstates)
        variants["fp64_plascc"]["removal_ms_per_step"] = round(r["ms_step"] - ms_step, 4)
        log(f"fp64 plascc step {r['ms_step']:.3f} ms")
    if compare:
        ksteps, kwarm = max(3, args.steps // 2), min(2, args.warmup)
        r = timed_steps(P, torch, ints, o, v, "bf16x3", ksteps, kwarm, guesses)
        variants["bf16x3"] = step_summary(r, flops, o, v, "bf16x3", nstates)
        variants["bf16x3"]["speedup_vs_fp64"] = round(ms_step / r["ms_step"], 3)
        log(f"bf16x3 step {r['ms_step']:.3f} ms")
        if not args.no_solves and nstates == 1:
            gate["fp64"] = timed_solve(P, torch, ints, o, v, "fp64", args.solve_tol)
            log(f"fp64 solve {gate['fp64']}")
            gate["bf16x3_refined"] = timed_solve(P, torch, ints, o, v, "bf16x3", args.solve_tol)
            log(f"bf16x3 solve {gate['bf16x3_refined']}")
    ints.close()
    torch.cuda.empty_cache()
    if compare:
        ints, _ = build_handle(P, torch, B, eps, o, args.vvvv, "fp32")
        r = timed_steps(P, torch, ints, o, v, "fp32", max(3, args.steps // 3), min(2, args.warmup), guesses)
        variants["fp32"] = step_summary(r, flops, o, v, "fp32", nstates)
        variants["fp32"]["speedup_vs_fp64"] = round(ms_step / r["ms_step"], 3)
        log(f"fp32 step {r['ms_step']:.3f} ms")
        if gate:
            gate["fp32_refined"] = timed_solve(P, torch, ints, o, v, "fp32", args.solve_tol)
            log(f"fp32 solve {gate['fp32_refined']}")
        ints.close()
        torch.cuda.empty_cache()
    del B
    if gate:
        ref = gate["fp64"]
        for name, g in gate.items():
            if name != "fp64":
                g["abs_dE_vs_fp64"] = abs(g["e_corr"] - ref["e_corr"])
                g["speedup_vs_fp64"] = round(ref["solve_s"] / g["solve_s"], 3)
            g["passes_gate"] = bool(g["converged"] and g.get("abs_dE_vs_fp64", 0.0) < 1e-6)
        for name in ("bf16x3", "fp32"):
            g = gate[f"{name}_refined"]
            variants[name].update(abs_dE_vs_fp64=g["abs_dE_vs_fp64"], max_abs_R=g["max_abs_R"],
                                  passes_gate=g["passes_gate"])
        out["precision_gate"] = dict(criterion=f"|R|_2 <= {args.solve_tol} on an FP64 residual; "
                                               "|E - E_FP64| < 1e-6 Eh against the FP64 GPU solve", **gate)
    if compare and args.workload != "o20v180q600":
        # the o20 v180 Q600 FP64 step with the full (ac|bd) block materialised (8.4 GB)
        wo = WORKLOADS["o20v180q600"]
        o2, v2, Q2 = wo["no"], wo["nv"], wo["naux"]
        B2, eps2 = make_system(o2, v2, Q2, wo["seed"], sigma=converging_sigma(v2, Q2))
        r = run_throughput(P, torch, B2, eps2, o2, v2, Q2, "full", "fp64", max(5, args.steps), args.warmup)
        variants["fp64_o20v180q600_full"] = step_summary(r, f_n6(o2, v2), o2, v2, "fp64")
        log(f"o20v180 fp64 step {r['ms_step']:.3f} ms")
        del B2
    if variants:
        out["variants"] = variants
    if not args.no_serve and nstates == 1:
        arrivals, reqs = serve_requests(args.requests)
        res = {}
        for name, pc in (("bf16x3_refined", P.ASCC_PREC_BF16X3), ("fp64", P.ASCC_PREC_FP64)):
            res[name] = run_serving(P, arrivals, reqs, pc, int(args.budget_gb * (1 << 30)), args.max_active,
                                    args.serve_tol, args.lowp_rnorm)
            log(f"serving {name}: {res[name]['solves_per_s']:.2f} solves/s")
        gate_serving(res)
        out["serving"] = {"workload": f"{args.requests} requests, Poisson 20/s, no U{{4..24}}, nv = 9 no, "
                                      f"naux = 3(no + nv), seeds 100..{99 + args.requests}",
                          "unit": "solves/s", "tol_rnorm": args.serve_tol, "hbm_budget_gb": args.budget_gb,
                          "max_active": args.max_active, "modes": res}
    if not args.no_counters:
        try:
            out["counters"] = run_counters(args)
            c = out["counters"]
            ring = c.get("ring_launch") or {}
            if ring.get("traffic_bytes") is not None:
                out["roofline"]["traffic"] = ring["traffic_bytes"]
                out["roofline"]["mfma_util"] = ring.get("mfma_util")
            out["fp64_step"]["mfma_util"] = (c.get("fp64_step") or {}).get("mfma_util")
            for name in ("bf16x3", "fp32"):
                if name in variants and f"{name}_step" in c:
                    variants[name]["mfma_util"] = c[f"{name}_step"]["mfma_util"]
        except Exception as exc:  # keep the measurement if the profiler is unavailable
            out["counters"] = {"error": str(exc)[:300]}
        if "serving" in out:
            try:
                out["serving"]["mfma_counters"] = run_serving_counters(SERVE_COUNTER_REQUESTS)
                for name, m in out["serving"]["mfma_counters"]["modes"].items():
                    log(f"serving {name}: MFMA busy {m['mfma_util']:.3f} over its kernels")
            except Exception as exc:
                out["serving"]["mfma_counters"] = {"error": str(exc)[:300]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(o, v, Q, seed, nstates)
    print(json.dumps(out), flush=True)


# ---- counters: rocprofv3 runs of this workload launched from here ----------------------------

COUNTER_PASSES = (
    ("fetch", ["FETCH_SIZE", "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU_MFMA_MOPS_F64",
               "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_BF16"]),
    ("write", ["WRITE_SIZE"]),
)
CALIB_BYTES = 1 << 30
RUN_T0 = time.perf_counter()  # the default run keeps its profiler passes within RUN_BUDGET_S of this
RUN_BUDGET_S = 480.0
SERVE_COUNTERS = ["SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU_MFMA_MOPS_F64",
                  "SQ_INSTS_VALU_MFMA_MOPS_BF16"]
SERVE_COUNTER_REQUESTS = 64


def run_serving_counters(nreq: int):
    """MFMA utilisation of the serving kernels: one rocprofv3 counter pass per mode over the first
    nreq requests of the serving stream.  The pass serialises the kernels, so the figure is that of
    the kernels themselves (busy cycles over their active cycles), not of the wall time."""
    import shutil

    exe = shutil.which("rocprofv3")
    if exe is None:
        raise RuntimeError("rocprofv3 not found")
    modes = {}
    for name, prec in (("bf16x3_refined", "bf16x3"), ("fp64", "fp64")):
        outdir = tempfile.mkdtemp(prefix=f"ascc_spmc_{prec}_")
        cmd = [exe, "--pmc", *SERVE_COUNTERS, "--output-format", "csv", "-d", outdir, "-o", "run", "--",
               sys.executable, os.path.abspath(__file__), "--serve", "--serve-precisions", prec,
               "--requests", str(nreq)]
        left = RUN_BUDGET_S - (time.perf_counter() - RUN_T0)
        if left < 60:
            raise RuntimeError(f"skipped: {RUN_BUDGET_S - left:.0f} s into the run, the {prec} pass would not fit")
        r = subprocess.run(["timeout", "-s", "KILL", str(int(min(150, left))), *cmd], capture_output=True, text=True,
                           cwd=tempfile.gettempdir(), env=dict(os.environ, TMPDIR=tempfile.gettempdir()))
        if r.returncode != 0:
            raise RuntimeError(f"serving counter pass {prec} failed (rc {r.returncode}): "
                               f"{(r.stderr or r.stdout)[-300:]}")
        rows = _read_counters(outdir)
        shutil.rmtree(outdir, ignore_errors=True)
        tot = {}
        for row in rows:
            for k, val in row["c"].items():
                tot[k] = tot.get(k, 0.0) + val
        act = tot.get("GRBM_GUI_ACTIVE", 0.0) / 8.0  # summed over the 8 XCDs
        modes[name] = {"mfma_util": tot.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (1024 * act) if act else None,
                       "mfma_flops_executed": {k.rsplit("_", 1)[-1]: v * 512 for k, v in tot.items() if "MOPS" in k},
                       "dispatches": len(rows)}
    return {"requests": nreq, "modes": modes,
            "method": "rocprofv3 --pmc " + " ".join(SERVE_COUNTERS) + f" over bench.py --serve --requests {nreq} "
                      "per mode, summed over its dispatches; MFMA utilisation = SQ_VALU_MFMA_BUSY_CYCLES / "
                      "(1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs), of the kernels (the pass serialises them)"}


def counter_child(args):
    """The profiled program: one FP64, one split-BF16x3 and one FP32 step of the workload (each after
    a warm-up step), then a plain device copy of CALIB_BYTES."""
    import torch

    import paper_2501_10515_amd as P

    wl = WORKLOADS[args.workload]
    o, v, Q, seed = wl["no"], wl["nv"], wl["naux"], wl["seed"]
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    ints, _ = build_handle(P, torch, B, eps, o, args.vvvv, "bf16x3")
    del B
    for prec in ("fp64", "bf16x3"):
        torch.cuda.synchronize()
        timed_steps(P, torch, ints, o, v, prec, 1, 1)
        torch.cuda.synchronize()
    ints.close()
    torch.cuda.empty_cache()
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    ints, _ = build_handle(P, torch, B, eps, o, args.vvvv, "fp32")
    del B
    timed_steps(P, torch, ints, o, v, "fp32", 1, 1)
    torch.cuda.synchronize()
    ints.close()
    torch.cuda.empty_cache()
    a = torch.empty(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    torch.cuda.synchronize()
    a.copy_(b)
    torch.cuda.synchronize()
    print("counter child done", flush=True)


def _read_counters(outdir):
    """Rows (dispatch id, kernel name, grid, {counter: value}) from rocprofv3's counter CSV."""
    import csv
    import glob

    files = glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise RuntimeError(f"no counter_collection.csv under {outdir}")
    rows = {}
    with open(files[0], newline="") as f:
        for rec in csv.DictReader(f):
            d = int(rec["Dispatch_Id"])
            r = rows.setdefault(d, {"kernel": rec["Kernel_Name"], "grid": int(rec.get("Grid_Size", 0) or 0),
                                    "wg": int(rec.get("Workgroup_Size", 0) or 0), "c": {}})
            r["c"][rec["Counter_Name"]] = r["c"].get(rec["Counter_Name"], 0.0) + float(rec["Counter_Value"])
    return [rows[k] for k in sorted(rows)]


def run_counters(args):
    """Two rocprofv3 counter passes (FETCH_SIZE with the MFMA counters, then WRITE_SIZE) over
    counter_child, each step's kernels told apart by dispatch order.  FETCH_SIZE and WRITE_SIZE are
    scaled by what they read for the calibration copy (CALIB_BYTES read and written)."""
    import shutil

    exe = shutil.which("rocprofv3")
    if exe is None:
        raise RuntimeError("rocprofv3 not found")
    passes = {}
    for name, counters in COUNTER_PASSES:
        outdir = tempfile.mkdtemp(prefix=f"ascc_pmc_{name}_")
        cmd = [exe, "--pmc", *counters, "--output-format", "csv", "-d", outdir, "-o", "run", "--",
               sys.executable, os.path.abspath(__file__), "--counter-child", "--workload", args.workload,
               "--vvvv", args.vvvv]
        t0 = time.perf_counter()
        r = subprocess.run(["timeout", "-s", "KILL", "150", *cmd], capture_output=True, text=True,
                           cwd=tempfile.gettempdir(), env=dict(os.environ, TMPDIR=tempfile.gettempdir()))
        if "counter child done" not in r.stdout:
            raise RuntimeError(f"rocprofv3 {name} pass failed (rc {r.returncode}): {(r.stderr or r.stdout)[-300:]}")
        passes[name] = _read_counters(outdir)
        shutil.rmtree(outdir, ignore_errors=True)
        print(f"counter pass {name}: {len(passes[name])} dispatches in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    return summarize_counters(passes, args)


def summarize_counters(passes, args):
    wl = WORKLOADS[args.workload]
    o, v = wl["no"], wl["nv"]
    fetch, write = passes["fetch"], passes["write"]
    if len(fetch) != len(write):
        raise RuntimeError("the two counter passes saw different dispatch sequences")
    calib_f = fetch[-1]["c"]["FETCH_SIZE"]
    calib_w = write[-1]["c"]["WRITE_SIZE"]
    kib = CALIB_BYTES / 1024
    fscale, wscale = kib / calib_f, kib / calib_w

    # the profiled program runs: the build, then warm-up + step in FP64, then warm-up + step in
    # split-BF16x3, then another build and warm-up + step in FP32, then the copy; every step ends
    # with the update's last kernel (update_stage3)
    seq = list(zip(fetch, write))
    ends = [k for k, (f, _) in enumerate(seq) if "update_stage3" in f["kernel"]]
    if len(ends) != 6:
        raise RuntimeError(f"expected 6 steps in the profiled program, found {len(ends)}")

    def agg(ks):
        busy = sum(seq[k][0]["c"].get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for k in ks)
        act = sum(seq[k][0]["c"].get("GRBM_GUI_ACTIVE", 0.0) for k in ks)
        mops = {p: sum(seq[k][0]["c"].get(f"SQ_INSTS_VALU_MFMA_MOPS_{p}", 0.0) for k in ks)
                for p in ("F64", "F32", "BF16")}
        byt = sum(seq[k][0]["c"]["FETCH_SIZE"] * fscale + seq[k][1]["c"]["WRITE_SIZE"] * wscale for k in ks) * 1024
        return {"mfma_util": round(busy / (act / XCDS * SIMDS), 4) if act else None,
                "mfma_flops_executed": {p: m * 512 for p, m in mops.items() if m}, "hbm_bytes": byt}

    out = {"calibration": {"copy_bytes": CALIB_BYTES, "fetch_scale": round(fscale, 4),
                           "write_scale": round(wscale, 4)},
           "method": "rocprofv3 --pmc, one FP64 and one split-BF16x3 step of this workload (each after a "
                     "warm-up step) in a child process; MFMA utilisation = SQ_VALU_MFMA_BUSY_CYCLES summed "
                     "over the 1024 SIMDs / (1024 x GPU-active cycles, GRBM_GUI_ACTIVE / 8 XCDs), over the "
                     "dispatches; mfma_flops_executed = SQ_INSTS_VALU_MFMA_MOPS_* x 512"}
    fp64_step = list(range(ends[0] + 1, ends[1] + 1))
    out["fp64_step"] = agg(fp64_step)
    out["bf16x3_step"] = agg(list(range(ends[2] + 1, ends[3] + 1)))
    fp32_first = ends[4] + 1  # the FP32 step follows its warm-up
    out["fp32_step"] = agg(list(range(fp32_first, ends[5] + 1)))
    # the pp-ladder launch of each step: its first contraction after the pair packing
    def ladder(rng, tag):
        ks = list(rng)
        pk = [k for k in ks if "pack_tpm" in seq[k][0]["kernel"]]
        if not pk:
            return None
        gm = [k for k in ks if k > pk[0] and "gemm_" in seq[k][0]["kernel"]]
        if not gm:
            return None
        # a ladder whose last row tile runs as tail tiles is two launches
        parts = gm[:2] if len(gm) > 1 and "_tail_" in seq[gm[1]][0]["kernel"] else gm[:1]
        a = agg(parts)
        name = seq[gm[0]][0]["kernel"]
        name = name[name.find("gemm_"):]
        return {"kernel": name[:max(name.find("("), 0) or len(name)][:60] + (" + tail" if len(parts) > 1 else ""),
                "traffic_bytes": a["hbm_bytes"],
                "mfma_util": a["mfma_util"], "algorithmic_flops": ladder_flops(o, v),
                "mfma_flops_executed": a["mfma_flops_executed"], "step": tag}
    for tag, rng in (("fp64", fp64_step), ("bf16x3", range(ends[2] + 1, ends[3] + 1)),
                     ("fp32", range(fp32_first, ends[5] + 1))):
        lad = ladder(rng, tag)
        if lad:
            out[f"{tag}_ladder_launch"] = lad
    # the ring launches of the FP64 step: its direct-to-LDS FP64 GEMM dispatches with the largest grid
    dma = [k for k in fp64_step if "gemm_f64_dma_kernel" in seq[k][0]["kernel"]]
    if dma:
        gmax = max(seq[k][0]["grid"] for k in dma)
        ring = [k for k in dma if seq[k][0]["grid"] == gmax]
        per = [agg([k]) for k in ring]
        name = seq[ring[0]][0]["kernel"]
        name = name[name.find("gemm_f64_dma_kernel"):]
        out["ring_launch"] = {"kernel": name[:name.find(">") + 1], "launches_per_step": len(ring),
                              "traffic_bytes": sum(p["hbm_bytes"] for p in per) / len(per),
                              "mfma_util": round(sum(p["mfma_util"] for p in per) / len(per), 4),
                              "algorithmic_flops": ring_flops(o, v),
                              "mfma_flops_executed": per[0]["mfma_flops_executed"]}
    return out


if __name__ == "__main__":
    main()
