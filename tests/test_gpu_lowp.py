"""Low-precision contractions (FP32, split-BF16x3) against the FP64 oracle, and FP64 refinement."""
import numpy as np
import pytest

from gen.synth_df import make_system, random_amplitudes, random_symmetric_fock

pytestmark = pytest.mark.gpu

# Error bounds relative to max|R| of the exact residual.  FP32 operands carry a relative
# rounding error u = 2^-24 each; BF16x3 products drop the lo*lo term (2^-16 relative) and keep
# hi/lo representation errors of 2^-17; both accumulate in FP32 within K chunks of 8192 (then FP64
# across chunks).  With sums of a few thousand terms of mixed sign the observed error stays well
# below sqrt(K)*u_eff times the largest term; the bounds below
# leave a factor of about ten over what is measured.
REL = {"fp32": 2e-6, "bf16x3": 4e-5}


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_10515_amd as P

    P.load_library()
    return P


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("mode", ["full", "packed"])
@pytest.mark.parametrize("o,v,Q,seed,full", [(2, 3, 8, 1, False), (5, 20, 60, 0, False), (7, 45, 37, 3, True),
                                             (9, 70, 130, 5, False)])
def test_lowp_residual_error_is_bounded(P, o, v, Q, seed, full, mode, prec):
    from oracle import cs_ccsd

    from .gpu_util import dev, gpu_residual

    print(f"case o={o} v={v} Q={Q} vvvv={mode} prec={prec}", flush=True)
    B, eps = make_system(o, v, Q, seed, sigma=0.1)
    fock = random_symmetric_fock(eps, 0.05, seed + 7) if full else np.diag(eps)
    t1, t2 = random_amplitudes(o, v, seed + 100, 0.05, 0.05)
    r1_ref, r2_ref = cs_ccsd.residual(B, fock, t1, t2)
    e_ref = cs_ccsd.energy(B, fock, t1, t2)
    pc = P.ASCC_PREC_FP32 if prec == "fp32" else P.ASCC_PREC_BF16X3
    vm = P.ASCC_VVVV_FULL if mode == "full" else P.ASCC_VVVV_PACKED
    ints = P.ascc_build_ints(dev(B), dev(fock if full else eps), o, precision=pc, vvvv_mode=vm)
    assert P.ascc_get_precision(ints) == pc
    r1, r2, e = gpu_residual(P, ints, t1, t2)
    scale = max(np.abs(r2_ref).max(), np.abs(r1_ref).max())
    err = max(np.abs(r1 - r1_ref).max(), np.abs(r2 - r2_ref).max())
    print(f"  max|dR| = {err:.3e}  (max|R| = {scale:.3e}, rel {err / scale:.2e})", flush=True)
    assert err <= REL[prec] * scale
    assert abs(e - e_ref) <= 1e-10  # the energy reduction is FP64 at the same amplitudes
    # the same handle switched to FP64 gives the exact residual
    P.ascc_set_precision(ints, P.ASCC_PREC_FP64)
    r1, r2, e = gpu_residual(P, ints, t1, t2)
    ints.close()
    assert max(np.abs(r1 - r1_ref).max(), np.abs(r2 - r2_ref).max()) <= 1e-10


@pytest.mark.parametrize("mode", ["full", "packed"])
def test_lowp_split_k_direct_to_lds_products(P, mode):
    """o10 v140: the ring pair (ov = 1400: 72 tiles of 256 x 256) is too small for one round, so the
    FP32 and split-BF16x3 direct-to-LDS kernels cut its K into two slices whose partial tiles
    (2 x 1400^2 doubles, within the split-K scratch) are summed in slice order; both residuals
    against the FP64 oracle."""
    from oracle import cs_ccsd

    from .gpu_util import dev, gpu_residual

    o, v, Q, seed = 10, 140, 200, 12
    B, eps = make_system(o, v, Q, seed, sigma=0.1)
    t1, t2 = random_amplitudes(o, v, seed + 100, 0.05, 0.05)
    r1_ref, r2_ref = cs_ccsd.residual(B, np.diag(eps), t1, t2)
    scale = max(np.abs(r2_ref).max(), np.abs(r1_ref).max())
    vm = P.ASCC_VVVV_FULL if mode == "full" else P.ASCC_VVVV_PACKED
    for prec, pc in (("fp32", P.ASCC_PREC_FP32), ("bf16x3", P.ASCC_PREC_BF16X3)):
        print(f"case o={o} v={v} Q={Q} vvvv={mode} prec={prec}", flush=True)
        ints = P.ascc_build_ints(dev(B), dev(eps), o, precision=pc, vvvv_mode=vm)
        r1, r2, _ = gpu_residual(P, ints, t1, t2)
        ints.close()
        err = max(np.abs(r1 - r1_ref).max(), np.abs(r2 - r2_ref).max())
        print(f"  max|dR| = {err:.3e}  (max|R| = {scale:.3e}, rel {err / scale:.2e})", flush=True)
        assert err <= REL[prec] * scale


def test_precision_switch_requires_low_precision_build(P):
    from .gpu_util import dev

    B, eps = make_system(2, 3, 8, 1)
    ints = P.ascc_build_ints(dev(B), dev(eps), 2)
    with pytest.raises(P.AsccError) as e:
        P.ascc_set_precision(ints, P.ASCC_PREC_BF16X3)
    assert e.value.code == P.ASCC_E_STATE
    ints.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_refined_solve_matches_fp64_oracle(P, prec):
    """Low-precision bulk iterations + FP64 refinement converge to the FP64 oracle's energy."""
    from oracle import cs_ccsd, solver

    from .gpu_util import dev

    o, v, Q = 5, 20, 60
    B, eps = make_system(o, v, Q, 0)
    fock = np.diag(eps)
    z1, z2 = np.zeros((o, v)), np.zeros((o, o, v, v))
    ref = solver.solve(lambda a, b: cs_ccsd.residual(B, fock, a, b), lambda a, b: cs_ccsd.energy(B, fock, a, b),
                       eps, z1, z2, maxiter=60, tol_rnorm=1e-8)
    pc = P.ASCC_PREC_FP32 if prec == "fp32" else P.ASCC_PREC_BF16X3
    ints = P.ascc_build_ints(dev(B), dev(eps), o, precision=pc, vvvv_mode=P.ASCC_VVVV_PACKED)
    t1, t2 = dev(z1), dev(z2)
    res = P.ascc_solve(ints, t1, t2, tol_rnorm=1e-8, maxiter=80, lowp_rnorm=1e-5)
    assert P.ascc_get_precision(ints) == pc  # restored
    ints.close()
    print(res, ref["E"], flush=True)
    assert res["converged"] and res["lowp_iterations"] >= 3
    assert abs(res["e_corr"] - ref["E"]) <= 1e-9


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("mode", ["full", "packed"])
def test_lowp_ladder_over_several_k_chunks(P, mode, prec):
    """o40 v130: the ladder product has M = T(o) = 820 rows per half and K = N = T(v) = 8515, so the
    split-BF16x3 contraction runs on its direct-to-LDS kernel (4 x 34 x 2 = 272 tiles of 256 x 256)
    and flushes its FP32 sums into the FP64 result twice (K chunks of 8192), as does the FP32 one on
    its direct-to-LDS kernel; in both, the last 52 rows of each half run as 64-row tail tiles in a
    launch of their own (3 x 34 x 2 full tiles in one round, then 68 tail tiles): the residual
    against the FP64 oracle."""
    from oracle import cs_ccsd

    from .gpu_util import dev, gpu_residual

    o, v, Q, seed = 40, 130, 200, 11
    print(f"case o={o} v={v} Q={Q} vvvv={mode} prec={prec}", flush=True)
    B, eps = make_system(o, v, Q, seed, sigma=0.1)
    t1, t2 = random_amplitudes(o, v, seed + 100, 0.02, 0.02)
    r1_ref, r2_ref = cs_ccsd.residual(B, np.diag(eps), t1, t2)
    pc = P.ASCC_PREC_FP32 if prec == "fp32" else P.ASCC_PREC_BF16X3
    vm = P.ASCC_VVVV_FULL if mode == "full" else P.ASCC_VVVV_PACKED
    ints = P.ascc_build_ints(dev(B), dev(eps), o, precision=pc, vvvv_mode=vm)
    r1, r2, e = gpu_residual(P, ints, t1, t2)
    scale = max(np.abs(r2_ref).max(), np.abs(r1_ref).max())
    err = max(np.abs(r1 - r1_ref).max(), np.abs(r2 - r2_ref).max())
    print(f"  max|dR| = {err:.3e}  (max|R| = {scale:.3e}, rel {err / scale:.2e})", flush=True)
    assert err <= REL[prec] * scale
    # the same handle switched to FP64 gives the exact residual
    P.ascc_set_precision(ints, P.ASCC_PREC_FP64)
    q1, q2, _ = gpu_residual(P, ints, t1, t2)
    ints.close()
    assert max(np.abs(q1 - r1_ref).max(), np.abs(q2 - r2_ref).max()) <= 1e-10 * max(1.0, scale)


@pytest.mark.slow
def test_mixed_precision_solves_meet_the_energy_gate_at_o40_v360(P):
    """The precision study's gate at o40 v360 Q1200 (seed 2, convergence-variant width): split-BF16x3
    and FP32 bulk iterations finished in FP64 land within |dE| < 1e-6 Eh of the FP64 GPU solve (the
    reference at this size), each converged to |R|_2 <= 1e-7 on an FP64 residual."""
    import torch

    from gen.synth_df import converging_sigma

    from .gpu_util import dev

    o, v, Q, seed = 40, 360, 1200, 2
    torch.cuda.empty_cache()  # the integral sets here take most of the device: start from free memory
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    dB, deps = dev(B), dev(eps)
    del B
    t1 = torch.zeros((o, v), dtype=torch.float64, device="cuda")
    t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    out = {}
    for prec in ("bf16x3", "fp32"):
        pc = P.ASCC_PREC_FP32 if prec == "fp32" else P.ASCC_PREC_BF16X3
        ints = P.ascc_build_ints(dB, deps, o, precision=pc, vvvv_mode=P.ASCC_VVVV_PACKED)
        if prec == "bf16x3":  # the FP64 reference on the same handle's FP64 operands
            P.ascc_set_precision(ints, P.ASCC_PREC_FP64)
            t1.zero_()
            t2.zero_()
            out["fp64"] = P.ascc_solve(ints, t1, t2, tol_rnorm=1e-7, maxiter=60)
            P.ascc_set_precision(ints, pc)
        t1.zero_()
        t2.zero_()
        out[prec] = P.ascc_solve(ints, t1, t2, tol_rnorm=1e-7, maxiter=60, lowp_rnorm=1e-7)
        ints.close()
        torch.cuda.empty_cache()
    for k, r in out.items():
        print(k, r, f"|dE| vs fp64 = {abs(r['e_corr'] - out['fp64']['e_corr']):.2e}", flush=True)
        assert r["converged"] and r["rnorm"] <= 1e-7
    for k in ("bf16x3", "fp32"):
        assert out[k]["lowp_iterations"] >= 5
        assert abs(out[k]["e_corr"] - out["fp64"]["e_corr"]) < 1e-6


TAIL_CHILD = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import paper_2501_10515_amd as P
from gen.synth_df import make_system, random_amplitudes
P.load_library()
o, v, Q, seed = 40, 130, 200, 11
B, eps = make_system(o, v, Q, seed, sigma=0.1)
t1, t2 = random_amplitudes(o, v, seed + 100, 0.02, 0.02)
dt1, dt2 = torch.from_numpy(t1).cuda(), torch.from_numpy(t2).cuda()
out = {}
for name, pc in (("fp32", P.ASCC_PREC_FP32), ("bf16x3", P.ASCC_PREC_BF16X3)):
    ints = P.ascc_build_ints(torch.from_numpy(B).cuda(), torch.from_numpy(eps).cuda(), o, precision=pc,
                             vvvv_mode=P.ASCC_VVVV_PACKED)
    r1, r2 = torch.empty_like(dt1), torch.empty_like(dt2)
    e = torch.empty(1, dtype=torch.float64, device="cuda")
    P.ascc_residual(ints, dt1, dt2, r1, r2, e)
    torch.cuda.synchronize()
    out[name + "_r1"], out[name + "_r2"], out[name + "_e"] = r1.cpu().numpy(), r2.cpu().numpy(), e.cpu().numpy()
    ints.close()
np.savez(sys.argv[2], **out)
print("done", flush=True)
"""


@pytest.mark.slow
def test_tail_tiles_give_the_full_launch_rows_bit_for_bit(P, tmp_path):
    """o40 v130 Q200, packed vvvv: the ladder's last row tile (52 of T(o) = 820 pair rows) runs as
    64-row tail tiles (3 x 34 x 2 full tiles fill one round, the 68 tail tiles a cheaper second
    one) in the FP32 and the split-BF16x3 contraction; with ASCC_NO_TAIL_TILES=1 (read once per
    process, so in children) it stays in the full-tile launch.  Both residuals and energies agree
    bit for bit, in both precisions."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = tmp_path / "tail_child.py"
    script.write_text(TAIL_CHILD)
    res = {}
    for knob in ("0", "1"):
        print(f"case: o40 v130 Q200 residuals, ASCC_NO_TAIL_TILES={knob}", flush=True)
        path = tmp_path / f"r{knob}.npz"
        r = subprocess.run([sys.executable, str(script), root, str(path)], capture_output=True, text=True,
                           timeout=240, env=dict(os.environ, ASCC_NO_TAIL_TILES=knob), cwd=root)
        assert r.returncode == 0, r.stderr[-2000:]
        res[knob] = np.load(path)
    for k in res["0"].files:  # the 64-bit patterns, so that even the sign of a zero must agree
        assert np.array_equal(res["0"][k].view(np.uint64), res["1"][k].view(np.uint64)), k
    assert np.abs(res["0"]["bf16x3_r2"]).max() > 1e-4
