"""Request server: continuous batching of independent solves; each result is the same alone and
in the mix, and matches the FP64 oracle."""
import time

import numpy as np
import pytest

from gen.synth_df import converging_sigma, make_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_10515_amd as P

    P.load_library()
    return P


def _requests():
    out = []
    for k, o in enumerate([3, 5, 4, 6, 2, 5]):
        v, Q = 4 * o, 3 * 5 * o
        B, eps = make_system(o, v, Q, 500 + k, sigma=converging_sigma(v, Q))
        out.append((o, B, eps))
    return out


def _serve(P, reqs, order, precision, gap=0.0, graphs=True, budget=2 << 30, max_active=8, tol_rnorm=1e-9,
           maxiter=200):
    srv = P.Server(budget, max_active=max_active, precision=precision, vvvv_mode=P.ASCC_VVVV_PACKED,
                   use_graphs=graphs, tol_rnorm=tol_rnorm, maxiter=maxiter, lowp_rnorm=1e-5)
    t0 = time.perf_counter()
    ids = {}
    pending = list(order)
    while True:
        now = time.perf_counter() - t0
        while pending and now >= gap * len(ids):
            k = pending.pop(0)
            o, B, eps = reqs[k][:3]
            state = reqs[k][3] if len(reqs[k]) > 3 else (-1, -1)  # (hole, particle[, plascc]) of a 1-CSF state
            ids[k] = srv.submit(B, eps, o, now, hole=state[0], particle=state[1],
                                plascc=len(state) > 2 and state[2])
        q, r, d = srv.step(now)
        if not pending and d == len(order):
            break
        if now > 120:
            raise TimeoutError("server did not finish")
    out = {k: srv.info(i) for k, i in ids.items()}
    srv.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_alone_equals_mixed_and_oracle(P, prec):
    from oracle import cs_ccsd, solver

    reqs = _requests()
    pc = P.ASCC_PREC_FP64 if prec == "fp64" else P.ASCC_PREC_BF16X3
    mixed = _serve(P, reqs, list(range(len(reqs))), pc, gap=0.0)
    for k in range(len(reqs)):
        alone = _serve(P, reqs, [k], pc)[k]
        m = mixed[k]
        print(k, prec, alone["e_corr"], m["e_corr"], alone["iterations"], m["iterations"], flush=True)
        assert alone["status"] == 0 and m["status"] == 0
        assert alone["iterations"] == m["iterations"]
        assert alone["e_corr"] == m["e_corr"]  # bitwise: no cross-request interaction
        o, B, eps = reqs[k]
        v = eps.size - o
        ref = solver.solve(lambda a, b: cs_ccsd.residual(B, np.diag(eps), a, b),
                           lambda a, b: cs_ccsd.energy(B, np.diag(eps), a, b), eps, np.zeros((o, v)),
                           np.zeros((o, o, v, v)), maxiter=200, tol_rnorm=1e-9)
        assert abs(m["e_corr"] - ref["E"]) <= 1e-8


@pytest.mark.parametrize("room", ["one", "two"])
def test_admission_respects_the_budget(P, room):
    """Footprint admission: at every moment the requests holding slab memory fit the budget.  With room
    for one request (the budget is below the two smallest footprints together) they run strictly one
    after another; with room for two, at most two overlap."""
    reqs = _requests()[:4]
    res = _serve(P, reqs, [0, 1, 2, 3], P.ASCC_PREC_FP64, budget=1 << 30)  # sizes from the server itself
    fp = sorted(r["bytes"] for r in res.values())
    budget = fp[-1] + (1 << 20) if room == "one" else fp[-1] + fp[-2] + (1 << 20)
    assert (fp[0] + fp[1] > budget) if room == "one" else (sum(fp[:3]) > budget)
    res = _serve(P, reqs, [0, 1, 2, 3], P.ASCC_PREC_FP64, budget=budget)
    assert all(r["status"] == 0 for r in res.values())
    iv = [(r["t_admit"], r["t_done"], r["bytes"]) for r in res.values()]
    for a, _, _ in iv:  # slab bytes held at each admission instant
        held = sum(b for a2, d2, b in iv if a2 <= a < d2)
        assert held <= budget
    if room == "one":
        iv.sort()
        for (a0, d0, _), (a1, d1, _) in zip(iv, iv[1:]):
            assert a1 >= d0
    else:
        assert max(sum(1 for a2, d2, _ in iv if a2 <= a < d2) for a, _, _ in iv) <= 2


def test_graph_replay_equals_direct_launches(P):
    reqs = _requests()[:2]
    a = _serve(P, reqs, [0, 1], P.ASCC_PREC_FP64, graphs=True)
    b = _serve(P, reqs, [0, 1], P.ASCC_PREC_FP64, graphs=False)
    for k in a:
        assert a[k]["e_corr"] == b[k]["e_corr"] and a[k]["iterations"] == b[k]["iterations"]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_served_excited_states_alone_equal_mixed_and_oracle(P, prec):
    """ASCC 1-CSF states (Hbar integral sets, T^P(0) guesses) served among ground-state requests."""
    from oracle import ascc, cs_ccsd, solver

    reqs = _requests()[:3]
    for o, v, Q, seed, hole, particle in [(3, 12, 36, 7, 2, 3), (6, 24, 72, 5, 5, 6)]:
        B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
        reqs.append((o, B, eps, (hole, particle)))
    pc = P.ASCC_PREC_FP64 if prec == "fp64" else P.ASCC_PREC_BF16X3
    mixed = _serve(P, reqs, list(range(len(reqs))), pc, tol_rnorm=1e-8, maxiter=400)
    for k in (3, 4):
        alone = _serve(P, reqs, [k], pc, tol_rnorm=1e-8, maxiter=400)[k]
        m = mixed[k]
        print(k, prec, m, flush=True)
        assert alone["status"] == 0 and m["status"] == 0
        assert (m["hole"], m["particle"]) == reqs[k][3]
        assert alone["iterations"] == m["iterations"] and alone["e_corr"] == m["e_corr"]
        o, B, eps, (hole, particle) = reqs[k]
        Bbar, fbar = ascc.transformed_inputs(B, eps, o, hole, particle)
        g1, g2 = ascc.initial_guess(o, eps.size - o, hole, particle)
        ref = solver.solve(lambda a, b: cs_ccsd.residual(Bbar, fbar, a, b),
                           lambda a, b: cs_ccsd.energy(Bbar, fbar, a, b), eps, g1, g2, maxiter=600,
                           tol_rnorm=1e-11)
        assert ref["converged"]
        assert abs(m["e_corr"] - ref["E"]) <= 2e-8
        assert abs(m["e_ref"] - ascc.reference_energy(Bbar, fbar, o)) <= 1e-10
    for k in range(3):  # the ground-state requests of the mix still match their own oracle
        o, B, eps = reqs[k]
        assert mixed[k]["status"] == 0 and mixed[k]["hole"] == -1
        assert abs(mixed[k]["e_ref"] - ascc.reference_energy(B, eps, o)) <= 1e-10


def test_served_plascc_state_matches_oracle(P):
    """A PLASCC state request (Sec. II.C) among ASCC and ground-state requests."""
    from oracle import ascc, plascc, solver

    o, v, Q, seed, hole, particle = 3, 12, 36, 7, 2, 3
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    reqs = _requests()[:2] + [(o, B, eps, (hole, particle)), (o, B, eps, (hole, particle, True))]
    res = _serve(P, reqs, [0, 1, 2, 3], P.ASCC_PREC_FP64, tol_rnorm=1e-8, maxiter=400)
    assert all(r["status"] == 0 for r in res.values())
    Bbar, fbar = ascc.transformed_inputs(B, eps, o, hole, particle)
    g1, g2 = ascc.initial_guess(o, v, hole, particle)
    ref = solver.solve(lambda a, b: plascc.residual(Bbar, fbar, a, b, hole, particle),
                       lambda a, b: plascc.energy(Bbar, fbar, a, b), eps, g1, g2, maxiter=600, tol_rnorm=1e-11)
    assert ref["converged"]
    print(res[3]["e_corr"], ref["E"], res[2]["e_corr"], flush=True)
    assert abs(res[3]["e_corr"] - ref["E"]) <= 2e-8
    assert abs(res[3]["e_corr"] - res[2]["e_corr"]) > 1e-4  # PLASCC differs from ASCC
    alone = _serve(P, reqs, [3], P.ASCC_PREC_FP64, tol_rnorm=1e-8, maxiter=400)[3]
    assert alone["iterations"] == res[3]["iterations"] and alone["e_corr"] == res[3]["e_corr"]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_same_size_requests_share_a_bucket_and_match_alone(P, prec):
    """Six requests of one shape (o4 v16 Q60, different integrals) arriving together run as slots of
    one bucket -- one batched launch per contraction for all of them -- and each result equals the
    request served alone bit for bit (the same kernels and summation order per slot), with two other
    shapes in the mix."""
    from oracle import cs_ccsd, solver

    reqs = []
    for k in range(6):
        B, eps = make_system(4, 16, 60, 700 + k, sigma=converging_sigma(16, 60))
        reqs.append((4, B, eps))
    for k, o in enumerate([3, 5]):
        v, Q = 4 * o, 15 * o
        B, eps = make_system(o, v, Q, 720 + k, sigma=converging_sigma(v, Q))
        reqs.append((o, B, eps))
    pc = P.ASCC_PREC_FP64 if prec == "fp64" else P.ASCC_PREC_BF16X3
    mixed = _serve(P, reqs, list(range(len(reqs))), pc, budget=4 << 30, max_active=16)
    buckets = {mixed[k]["bucket"] for k in range(6)}
    assert len(buckets) == 1 and sorted(mixed[k]["slot"] for k in range(6)) == list(range(6))
    assert all(mixed[k]["bucket"] not in buckets for k in (6, 7))
    for k in range(len(reqs)):
        alone = _serve(P, reqs, [k], pc, budget=4 << 30)[k]
        m = mixed[k]
        print(k, prec, m["e_corr"], alone["e_corr"], m["iterations"], m["lowp_iterations"], flush=True)
        assert alone["status"] == 0 and m["status"] == 0
        assert alone["iterations"] == m["iterations"] and alone["lowp_iterations"] == m["lowp_iterations"]
        assert alone["e_corr"] == m["e_corr"]
    o, B, eps = reqs[2]
    ref = solver.solve(lambda a, b: cs_ccsd.residual(B, np.diag(eps), a, b),
                       lambda a, b: cs_ccsd.energy(B, np.diag(eps), a, b), eps, np.zeros((o, 16)),
                       np.zeros((o, o, 16, 16)), maxiter=200, tol_rnorm=1e-9)
    assert abs(mixed[2]["e_corr"] - ref["E"]) <= 1e-8


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_thirty_two_requests_match_the_oracle(P, prec):
    """A stream of 32 requests of five shapes (o2-o6, v = 4o, Q = 15o; up to eight of one shape),
    arriving together into at most 16 in flight: every one converges, several share
    buckets, every energy is within 1e-8 Eh of the oracle's solve of the same system, and four of
    them equal the request served alone bit for bit."""
    from oracle import cs_ccsd, solver

    sizes = [2, 3, 4, 5, 6, 4, 3, 5, 4, 2, 6, 4, 3, 5, 4, 3, 2, 4, 5, 3, 6, 4, 3, 5, 2, 4, 3, 5, 4, 6, 3, 5]
    reqs = []
    for k, o in enumerate(sizes):
        v, Q = 4 * o, 15 * o
        B, eps = make_system(o, v, Q, 800 + k, sigma=converging_sigma(v, Q))
        reqs.append((o, B, eps))
    pc = P.ASCC_PREC_FP64 if prec == "fp64" else P.ASCC_PREC_BF16X3
    mixed = _serve(P, reqs, list(range(len(reqs))), pc, budget=4 << 30, max_active=16)
    assert all(mixed[k]["status"] == 0 for k in range(len(reqs)))
    assert max(mixed[k]["slot"] for k in range(len(reqs))) >= 2  # some bucket held three or more slots
    for k, (o, B, eps) in enumerate(reqs):
        v = eps.size - o
        ref = solver.solve(lambda a, b: cs_ccsd.residual(B, np.diag(eps), a, b),
                           lambda a, b: cs_ccsd.energy(B, np.diag(eps), a, b), eps, np.zeros((o, v)),
                           np.zeros((o, o, v, v)), maxiter=200, tol_rnorm=1e-9)
        print(k, o, prec, mixed[k]["e_corr"], ref["E"], mixed[k]["bucket"], mixed[k]["slot"], flush=True)
        assert abs(mixed[k]["e_corr"] - ref["E"]) <= 1e-8
    for k in (0, 7, 18, 29):
        alone = _serve(P, reqs, [k], pc, budget=4 << 30)[k]
        assert alone["iterations"] == mixed[k]["iterations"] and alone["e_corr"] == mixed[k]["e_corr"]
