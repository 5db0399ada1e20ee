"""HIP residual / energy / update / solve against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from gen.synth_df import converging_sigma, make_system, random_amplitudes, random_symmetric_fock

pytestmark = pytest.mark.gpu

TOL = 1e-10  # per-element absolute tolerance for the FP64 path


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_10515_amd as P

    P.load_library()
    return P


def _case(o, v, Q, seed, full_fock, sigma=0.1, amp=0.05):
    B, eps = make_system(o, v, Q, seed, sigma=sigma)
    fock = random_symmetric_fock(eps, 0.05, seed + 7) if full_fock else np.diag(eps)
    t1, t2 = random_amplitudes(o, v, seed + 100, amp, amp)
    return B, eps, fock, t1, t2


SHAPES = [
    (1, 1, 1, 11, False),   # smallest system
    (2, 3, 8, 1, False),
    (3, 5, 12, 2, True),    # non-canonical, non-HF Fock matrix
    (5, 20, 60, 0, False),  # the o5 v20 Q60 shape
    (7, 45, 37, 3, True),   # ragged against every tile size
    (4, 70, 150, 4, False),
    (9, 33, 130, 5, True),
    (19, 24, 60, 6, False), # 190 pair rows: one 208-row ladder tile
    (21, 22, 60, 7, True),  # 231 pair rows: one 240-row ladder tile
]


@pytest.mark.parametrize("mode", ["full", "packed"])
@pytest.mark.parametrize("o,v,Q,seed,full", SHAPES)
def test_residual_and_energy_match_oracle(P, o, v, Q, seed, full, mode):
    from oracle import cs_ccsd

    from .gpu_util import dev, gpu_residual

    print(f"case o={o} v={v} Q={Q} seed={seed} full_fock={full} vvvv={mode}", flush=True)
    B, eps, fock, t1, t2 = _case(o, v, Q, seed, full)
    r1_ref, r2_ref = cs_ccsd.residual(B, fock, t1, t2)
    e_ref = cs_ccsd.energy(B, fock, t1, t2)
    vm = P.ASCC_VVVV_FULL if mode == "full" else P.ASCC_VVVV_PACKED
    ints = P.ascc_build_ints(dev(B), dev(fock if full else eps), o, vvvv_mode=vm)
    r1, r2, e = gpu_residual(P, ints, t1, t2)
    ints.close()
    assert np.abs(r1 - r1_ref).max() <= TOL
    assert np.abs(r2 - r2_ref).max() <= TOL
    assert abs(e - e_ref) <= TOL
    # closed-shell pair symmetry holds by construction
    assert np.abs(r2 - r2.transpose(1, 0, 3, 2)).max() <= TOL


def test_update_steps_match_oracle_diis(P):
    """Four Jacobi+DIIS steps on fixed residuals equal the oracle's DIIS bookkeeping."""
    import torch

    from oracle.solver import DIIS, denominators

    from .gpu_util import dev, host

    o, v, Q = 4, 11, 20
    B, eps, fock, t1, t2 = _case(o, v, Q, 21, False)
    ints = P.ascc_build_ints(dev(B), dev(eps), o)
    diis = P.ascc_diis_create(ints, 3, 1)
    d1, d2 = denominators(eps, o)
    ref = DIIS(3)
    dt1, dt2 = dev(t1), dev(t2)
    stats = torch.empty(8, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(5)
    for it in range(6):
        r1 = rng.normal(0, 0.01, (o, v))
        x = rng.normal(0, 0.01, (o, o, v, v))
        r2 = 0.5 * (x + x.transpose(1, 0, 3, 2))
        e = np.array([-0.1 * it])
        P.ascc_update(ints, diis, dt1, dt2, dev(r1), dev(r2), dev(e), stats)
        # oracle
        s1, s2 = r1 / d1, r2 / d2
        t1, t2 = t1 + s1, t2 + s2
        if it >= 1:
            ref.push(np.concatenate([t1.ravel(), t2.ravel()]), np.concatenate([s1.ravel(), s2.ravel()]))
            xx, _ = ref.extrapolate()
            if xx is not None:
                t1 = xx[: o * v].reshape(o, v)
                t2 = xx[o * v:].reshape(o, o, v, v)
        torch.cuda.synchronize()
        st = host(stats)
        assert np.abs(host(dt1) - t1).max() <= 1e-12
        assert np.abs(host(dt2) - t2).max() <= 1e-12
        assert st[3] == pytest.approx(np.sqrt((r1 ** 2).sum() + (r2 ** 2).sum()), rel=1e-13)
        assert st[2] == pytest.approx(max(np.abs(r1).max(), np.abs(r2).max()), rel=1e-15)
        assert st[0] == e[0]
        assert int(st[4]) == len(ref.vecs)
    diis.close()
    ints.close()


def test_solve_matches_oracle_o5v20q60(P):
    from oracle import cs_ccsd, solver

    from .gpu_util import dev, host

    o, v, Q = 5, 20, 60
    B, eps = make_system(o, v, Q, 0)
    fock = np.diag(eps)
    z1, z2 = np.zeros((o, v)), np.zeros((o, o, v, v))
    ref = solver.solve(lambda a, b: cs_ccsd.residual(B, fock, a, b), lambda a, b: cs_ccsd.energy(B, fock, a, b),
                       eps, z1, z2, maxiter=60, tol_rnorm=1e-8)
    assert ref["converged"]
    ints = P.ascc_build_ints(dev(B), dev(eps), o)
    t1, t2 = dev(z1), dev(z2)
    res = P.ascc_solve(ints, t1, t2, tol_rnorm=1e-8, maxiter=60)
    ints.close()
    assert res["converged"]
    assert res["rnorm"] <= 1e-8
    assert abs(res["e_corr"] - ref["E"]) <= 1e-9
    assert np.abs(host(t2) - ref["t2"]).max() <= 1e-8


@pytest.mark.slow
def test_residual_parity_o20v180q600_full_size():
    """Full-size residual (the o20 v180 Q600 workload, literal generator) against the oracle, both vvvv modes."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_10515_amd as P
    from oracle import cs_ccsd

    from .gpu_util import dev, gpu_residual

    o, v, Q = 20, 180, 600
    B, eps = make_system(o, v, Q, 1)
    t1, t2 = random_amplitudes(o, v, 77, 0.01, 0.01)
    fock = np.diag(eps)
    r1_ref, r2_ref = cs_ccsd.residual(B, fock, t1, t2)
    e_ref = cs_ccsd.energy(B, fock, t1, t2)
    scale = max(1.0, np.abs(r2_ref).max())
    for vm in (P.ASCC_VVVV_FULL, P.ASCC_VVVV_PACKED):
        print(f"o20v180q600 vvvv_mode={vm}", flush=True)
        ints = P.ascc_build_ints(dev(B), dev(eps), o, vvvv_mode=vm)
        r1, r2, e = gpu_residual(P, ints, t1, t2)
        ints.close()
        torch.cuda.empty_cache()
        assert np.abs(r1 - r1_ref).max() <= TOL * scale
        assert np.abs(r2 - r2_ref).max() <= TOL * scale
        assert abs(e - e_ref) <= TOL * max(1.0, abs(e_ref))


@pytest.mark.slow
def test_residual_parity_direct_to_lds_paths_ragged():
    """o17 v132 Q400 against the oracle, both vvvv modes: sized so that every large contraction takes
    the direct-to-LDS FP64 path with ragged tiles (rings ov = 2244 = 11 x 192 + 132; ladder
    T(o) = 153 rows in 224-row tiles and T(v) = 8778 = 68 x 128 + 74 columns; W/Z split over K with
    o^2 = 289 rows; G1/G3 with K = Q; N_Q split over K)."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_10515_amd as P
    from oracle import cs_ccsd

    from .gpu_util import dev, gpu_residual

    o, v, Q = 17, 132, 400
    B, eps = make_system(o, v, Q, 21, sigma=converging_sigma(v, Q))
    t1, t2 = random_amplitudes(o, v, 78, 0.02, 0.02)
    fock = np.diag(eps)
    r1_ref, r2_ref = cs_ccsd.residual(B, fock, t1, t2)
    e_ref = cs_ccsd.energy(B, fock, t1, t2)
    scale = max(1.0, np.abs(r2_ref).max())
    for vm in (P.ASCC_VVVV_FULL, P.ASCC_VVVV_PACKED):
        print(f"o17v132q400 vvvv_mode={vm}", flush=True)
        ints = P.ascc_build_ints(dev(B), dev(eps), o, vvvv_mode=vm)
        r1, r2, e = gpu_residual(P, ints, t1, t2)
        ints.close()
        torch.cuda.empty_cache()
        assert np.abs(r1 - r1_ref).max() <= TOL * scale
        assert np.abs(r2 - r2_ref).max() <= TOL * scale
        assert abs(e - e_ref) <= TOL * max(1.0, abs(e_ref))
