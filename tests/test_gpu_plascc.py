"""PLASCC on the GPU (ascc_set_plascc), through the C ABI, against the oracle (oracle/plascc.py,
itself pinned to brute-force projections with the mixed doubles taken in the spin-orbital basis)."""
import numpy as np
import pytest

from gen.synth_df import converging_sigma, make_system, random_amplitudes, random_symmetric_fock

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_10515_amd as P

    P.load_library()
    return P


SHAPES = [
    (2, 3, 8, 1, 0, 3, False),    # smallest with a hole below the top
    (3, 5, 12, 2, 2, 3, True),    # non-canonical Fock matrix
    (1, 4, 9, 4, 0, 1, False),    # o = 1: the primary set is one whole occupied row block
    (5, 20, 60, 0, 4, 5, False),  # HOMO -> LUMO at o5 v20 Q60
    (7, 45, 37, 3, 6, 9, True),   # ragged against every tile size
    (4, 70, 150, 4, 1, 73, False),  # particle = the last virtual
]


@pytest.mark.parametrize("transformed", [True, False])
@pytest.mark.parametrize("mode", ["full", "packed"])
@pytest.mark.parametrize("o,v,Q,seed,hole,particle,full", SHAPES)
def test_plascc_residual_matches_oracle(P, o, v, Q, seed, hole, particle, full, mode, transformed):
    from oracle import ascc, plascc

    from .gpu_util import dev, gpu_residual

    print(f"case o={o} v={v} Q={Q} seed={seed} {hole}->{particle} full={full} vvvv={mode} hbar={transformed}",
          flush=True)
    B, eps = make_system(o, v, Q, seed, sigma=0.1)
    fock = random_symmetric_fock(eps, 0.05, seed + 7) if full else np.diag(eps)
    if transformed:
        Bx, fx = ascc.transformed_inputs(B, fock, o, hole, particle)
    else:
        Bx, fx = B, fock
    t1, t2 = random_amplitudes(o, v, seed + 100, 0.05, 0.05)
    g1, g2 = ascc.initial_guess(o, v, hole, particle)
    t1, t2 = t1 + g1, t2 + g2
    r1_ref, r2_ref = plascc.residual(Bx, fx, t1, t2, hole, particle)
    e_ref = plascc.energy(Bx, fx, t1, t2)
    vm = P.ASCC_VVVV_FULL if mode == "full" else P.ASCC_VVVV_PACKED
    src = dev(fock if full else eps)
    if transformed:
        ints = P.ascc_build_ints_hbar(dev(B), src, o, hole, particle, vvvv_mode=vm)
    else:
        ints = P.ascc_build_ints(dev(B), src, o, vvvv_mode=vm)
    c1, c2, _ = gpu_residual(P, ints, t1, t2)  # the full equations first
    P.ascc_set_plascc(ints, hole, particle)
    r1, r2, e = gpu_residual(P, ints, t1, t2)
    # switched off again: the full residual, bit for bit
    P.ascc_set_plascc(ints, -1)
    d1, d2, _ = gpu_residual(P, ints, t1, t2)
    ints.close()
    scale = max(1.0, np.abs(r2_ref).max())
    assert np.abs(r1 - r1_ref).max() <= TOL * scale
    assert np.abs(r2 - r2_ref).max() <= TOL * scale
    assert abs(e - e_ref) <= TOL * scale
    assert np.abs(r2 - c2).max() > 1e-6  # the removal did something
    assert np.array_equal(c1, d1) and np.array_equal(c2, d2)
    assert np.abs(r2 - r2.transpose(1, 0, 3, 2)).max() <= 1e-14 * scale


REL = {"fp32": 2e-6, "bf16x3": 4e-5}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("o,v,Q,seed,hole,particle,full", [SHAPES[1], SHAPES[4]])
def test_plascc_low_precision_residual_error_is_bounded(P, o, v, Q, seed, hole, particle, full, prec):
    from oracle import ascc, plascc

    from .gpu_util import dev, gpu_residual

    print(f"case o={o} v={v} Q={Q} seed={seed} {hole}->{particle} {prec}", flush=True)
    B, eps = make_system(o, v, Q, seed, sigma=0.1)
    fock = random_symmetric_fock(eps, 0.05, seed + 7) if full else np.diag(eps)
    Bbar, fbar = ascc.transformed_inputs(B, fock, o, hole, particle)
    t1, t2 = random_amplitudes(o, v, seed + 100, 0.05, 0.05)
    g1, g2 = ascc.initial_guess(o, v, hole, particle)
    t1, t2 = t1 + g1, t2 + g2
    r1_ref, r2_ref = plascc.residual(Bbar, fbar, t1, t2, hole, particle)
    pc = P.ASCC_PREC_FP32 if prec == "fp32" else P.ASCC_PREC_BF16X3
    ints = P.ascc_build_ints_hbar(dev(B), dev(fock if full else eps), o, hole, particle, precision=pc,
                                  vvvv_mode=P.ASCC_VVVV_PACKED)
    P.ascc_set_plascc(ints, hole, particle)
    r1, r2, _ = gpu_residual(P, ints, t1, t2)
    ints.close()
    scale = max(np.abs(r2_ref).max(), np.abs(r1_ref).max())
    err = max(np.abs(r1 - r1_ref).max(), np.abs(r2 - r2_ref).max())
    print(f"  max|dR| = {err:.3e}  (max|R| = {scale:.3e}, rel {err / scale:.2e})", flush=True)
    assert err <= REL[prec] * scale


def test_plascc_batched_residual_equals_single(P):
    import torch

    from oracle import ascc

    from .gpu_util import dev

    o, v, Q, seed, hole, particle = 4, 30, 60, 11, 2, 6
    B, eps = make_system(o, v, Q, seed, sigma=0.1)
    ints = P.ascc_build_ints_hbar(dev(B), dev(eps), o, hole, particle, vvvv_mode=P.ASCC_VVVV_PACKED)
    P.ascc_set_plascc(ints, hole, particle)
    g1, g2 = ascc.initial_guess(o, v, hole, particle)
    states = []
    for k in range(3):
        t1, t2 = random_amplitudes(o, v, seed + k, 0.05, 0.05)
        states.append((dev(t1 + g1), dev(t2 + g2)))
    P.ascc_batch_reserve(ints, 3)
    r1s = [torch.empty_like(s[0]) for s in states]
    r2s = [torch.empty_like(s[1]) for s in states]
    e = torch.empty(3, dtype=torch.float64, device="cuda")
    P.ascc_residual_batch(ints, [s[0] for s in states], [s[1] for s in states], r1s, r2s, e)
    for k, (t1, t2) in enumerate(states):
        a1, a2 = torch.empty_like(t1), torch.empty_like(t2)
        ek = torch.empty(1, dtype=torch.float64, device="cuda")
        P.ascc_residual(ints, t1, t2, a1, a2, ek)
        torch.cuda.synchronize()
        assert torch.equal(a1, r1s[k]) and torch.equal(a2, r2s[k]) and float(ek) == float(e[k])
    ints.close()


# systems whose PLASCC excited-state iteration converges from T^P(0) in the oracle
SOLVES = [(3, 12, 36, 7, 2, 3), (6, 24, 72, 5, 5, 6)]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("o,v,Q,seed,hole,particle", SOLVES)
def test_plascc_excited_and_ground_solves_match_oracle(P, o, v, Q, seed, hole, particle, prec):
    import torch

    from oracle import ascc, plascc, solver

    print(f"solve o={o} v={v} Q={Q} seed={seed} {hole}->{particle} {prec}", flush=True)
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    f = np.diag(eps)
    Bbar, fbar = ascc.transformed_inputs(B, eps, o, hole, particle)
    g1, g2 = ascc.initial_guess(o, v, hole, particle)
    ref_x = solver.solve(lambda a, b: plascc.residual(Bbar, fbar, a, b, hole, particle),
                         lambda a, b: plascc.energy(Bbar, fbar, a, b), eps, g1, g2, maxiter=600, tol_rnorm=1e-11)
    ref_g = solver.solve(lambda a, b: plascc.residual(B, f, a, b, hole, particle),
                         lambda a, b: plascc.energy(B, f, a, b), eps, 0 * g1, 0 * g2, maxiter=300, tol_rnorm=1e-11)
    assert ref_x["converged"] and ref_g["converged"]
    pc = P.ASCC_PREC_FP64 if prec == "fp64" else P.ASCC_PREC_BF16X3
    lowp = 1e-6 if prec != "fp64" else 0.0
    dB, deps = torch.from_numpy(B).cuda(), torch.from_numpy(eps).cuda()
    t1 = torch.empty((o, v), dtype=torch.float64, device="cuda")
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device="cuda")
    ints = P.ascc_build_ints_hbar(dB, deps, o, hole, particle, precision=pc, vvvv_mode=P.ASCC_VVVV_PACKED)
    P.ascc_set_plascc(ints, hole, particle)
    P.ascc_initial_guess(t1, t2, hole, particle)
    rx = P.ascc_solve(ints, t1, t2, tol_rnorm=1e-8, maxiter=400, lowp_rnorm=lowp, raise_on_not_converged=False)
    ex = P.ascc_reference_energy(ints) + rx["e_corr"]
    ints.close()
    print(prec, "excited", rx, flush=True)
    assert rx["converged"]
    assert abs(rx["e_corr"] - ref_x["E"]) <= 2e-8
    assert np.abs(t2.cpu().numpy() - ref_x["t2"]).max() <= 1e-7
    ints = P.ascc_build_ints(dB, deps, o, precision=pc, vvvv_mode=P.ASCC_VVVV_PACKED)
    P.ascc_set_plascc(ints, hole, particle)
    t1.zero_()
    t2.zero_()
    rg = P.ascc_solve(ints, t1, t2, tol_rnorm=1e-8, maxiter=200, lowp_rnorm=lowp, raise_on_not_converged=False)
    eg = P.ascc_reference_energy(ints) + rg["e_corr"]
    ints.close()
    print(prec, "ground", rg, "excitation", ex - eg, flush=True)
    assert rg["converged"]
    assert abs(rg["e_corr"] - ref_g["E"]) <= 2e-8
    omega_ref = (ascc.reference_energy(Bbar, fbar, o) + ref_x["E"]) - (ascc.reference_energy(B, f, o) + ref_g["E"])
    assert abs((ex - eg) - omega_ref) <= 4e-8


@pytest.mark.slow
def test_ascc_and_plascc_residuals_at_full_size(P):
    """The o20 v180 Q600 workload with the full vvvv block, state 19 -> 20 (HOMO -> LUMO): the
    Hbar residual and the PLASCC residual against the oracle.  The crosses have m = o + v - 1 = 199
    rows, so every cross slab of the removal spans more than one tile."""
    import torch

    from oracle import ascc, cs_ccsd, plascc

    from .gpu_util import dev, gpu_residual

    o, v, Q, hole, particle = 20, 180, 600, 19, 20
    B, eps = make_system(o, v, Q, 1, sigma=converging_sigma(v, Q))
    Bbar, fbar = ascc.transformed_inputs(B, eps, o, hole, particle)
    t1, t2 = random_amplitudes(o, v, 79, 0.01, 0.01)
    g1, g2 = ascc.initial_guess(o, v, hole, particle)
    t1, t2 = t1 + g1, t2 + g2
    ints = P.ascc_build_ints_hbar(dev(B), dev(eps), o, hole, particle, vvvv_mode=P.ASCC_VVVV_FULL)
    a1, a2, ea = gpu_residual(P, ints, t1, t2)
    P.ascc_set_plascc(ints, hole, particle)
    p1, p2, ep = gpu_residual(P, ints, t1, t2)
    ints.close()
    torch.cuda.empty_cache()
    print("GPU residuals done; oracle ...", flush=True)
    r1_ref, r2_ref = cs_ccsd.residual(Bbar, fbar, t1, t2)
    e_ref = cs_ccsd.energy(Bbar, fbar, t1, t2)
    scale = max(1.0, np.abs(r2_ref).max())
    assert np.abs(a1 - r1_ref).max() <= TOL * scale
    assert np.abs(a2 - r2_ref).max() <= TOL * scale
    assert abs(ea - e_ref) <= TOL * max(1.0, abs(e_ref))
    c = plascc.mixed_quadratic(Bbar, fbar, t1, t2, hole, particle)
    print(f"max|c| = {np.abs(c).max():.3e}", flush=True)
    assert np.abs(c).max() > 1e-6
    assert np.array_equal(p1, a1) and ep == ea  # the singles and the energy keep every term
    assert np.abs(p2 - (r2_ref - c)).max() <= TOL * scale
    # the split-BF16x3 step that the bench times beside it, within the low-precision bound
    ints = P.ascc_build_ints_hbar(dev(B), dev(eps), o, hole, particle, precision=P.ASCC_PREC_BF16X3,
                                  vvvv_mode=P.ASCC_VVVV_FULL)
    P.ascc_set_plascc(ints, hole, particle)
    q1, q2, _ = gpu_residual(P, ints, t1, t2)
    ints.close()
    torch.cuda.empty_cache()
    rs = max(np.abs(r2_ref - c).max(), np.abs(r1_ref).max())
    err = max(np.abs(q1 - r1_ref).max(), np.abs(q2 - (r2_ref - c)).max())
    print(f"bf16x3: max|dR| = {err:.3e} (max|R| = {rs:.3e}, rel {err / rs:.2e})", flush=True)
    assert err <= REL["bf16x3"] * rs


def test_plascc_workspace_form_equals_the_allocating_form(P):
    """ascc_set_plascc_ws (buffers carved from a caller workspace filled with garbage, cleared on the
    stream) gives the residual of ascc_set_plascc bit for bit, on two primaries in a row."""
    import torch

    from .gpu_util import dev, gpu_residual

    o, v, Q, seed = 7, 45, 37, 3
    B, eps = make_system(o, v, Q, seed, sigma=0.1)
    t1, t2 = random_amplitudes(o, v, seed + 100, 0.05, 0.05)
    a = P.ascc_build_ints(dev(B), dev(eps), o, vvvv_mode=P.ASCC_VVVV_PACKED)
    b = P.ascc_build_ints(dev(B), dev(eps), o, vvvv_mode=P.ASCC_VVVV_PACKED)
    nbytes = P.ascc_plascc_workspace_bytes(o, v, Q)
    ws = torch.full((nbytes // 8,), float("nan"), dtype=torch.float64, device="cuda")
    for hole, particle in [(6, 9), (2, 7 + 44)]:
        P.ascc_set_plascc(a, hole, particle)
        P.ascc_set_plascc_ws(b, hole, particle, ws)
        ra, rb = gpu_residual(P, a, t1, t2), gpu_residual(P, b, t1, t2)
        assert np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1]) and ra[2] == rb[2]
    with pytest.raises(P.AsccError) as exc:  # one byte short
        c = P.ascc_build_ints(dev(B), dev(eps), o, vvvv_mode=P.ASCC_VVVV_PACKED)
        P.ascc_set_plascc_ws(c, 6, 9, ws[: (nbytes - 8) // 8])
    assert exc.value.code == P.ASCC_E_NOMEM
    a.close()
    b.close()


def test_served_plascc_request_footprint_is_exact(P):
    """A PLASCC request's slab share is its integral set, DIIS state, amplitudes, staging and the
    PLASCC buffers, each as the workspace queries report them: nothing is allocated beside the slab."""
    import time

    o, v, Q, seed, hole, particle = 3, 12, 36, 7, 2, 3
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    srv = P.Server(1 << 30, max_active=2, precision=P.ASCC_PREC_FP64, vvvv_mode=P.ASCC_VVVV_PACKED, tol_rnorm=1e-8,
                   maxiter=400)
    ids = [srv.submit(B, eps, o, 0.0, hole=hole, particle=particle),
           srv.submit(B, eps, o, 0.0, hole=hole, particle=particle, plascc=True)]
    t0 = time.perf_counter()
    while srv.step(time.perf_counter() - t0)[2] < 2:
        assert time.perf_counter() - t0 < 60
    plain, pl = srv.info(ids[0]), srv.info(ids[1])
    srv.close()
    assert plain["status"] == 0 and pl["status"] == 0
    extra = P.ascc_plascc_workspace_bytes(o, v, Q)
    assert pl["bytes"] - plain["bytes"] == (extra + 255) // 256 * 256
    ib, db = P.ascc_workspace_bytes(o, v, Q, P.ASCC_PREC_FP64, P.ASCC_VVVV_PACKED, 8)
    n = o + v

    def al(x):
        return (x + 255) // 256 * 256

    expect = al(ib) + al(db) + 2 * al(8 * o * v) + 2 * al(8 * o * o * v * v) + al(8) + al(8 * n) + al(8 * Q * n * n)
    assert plain["bytes"] == expect
