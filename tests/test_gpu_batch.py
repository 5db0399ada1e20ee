"""Several amplitude sets on one integral set: one batched ladder launch, per-state results
identical to the single-state residual (bitwise) and to the oracle."""
import numpy as np
import pytest

from gen.synth_df import make_system, random_amplitudes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_10515_amd as P

    P.load_library()
    return P


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("mode", ["full", "packed"])
@pytest.mark.parametrize("o,v,Q,S", [(3, 7, 15, 3), (6, 40, 90, 5)])
def test_batch_equals_alone_bitwise(P, o, v, Q, S, mode, prec):
    import torch

    from oracle import cs_ccsd

    from .gpu_util import dev, gpu_residual, host

    print(f"case o={o} v={v} Q={Q} S={S} vvvv={mode} prec={prec}", flush=True)
    B, eps = make_system(o, v, Q, 42, sigma=0.1)
    amps = [random_amplitudes(o, v, 300 + k, 0.05, 0.05) for k in range(S)]
    pc = P.ASCC_PREC_FP64 if prec == "fp64" else P.ASCC_PREC_BF16X3
    vm = P.ASCC_VVVV_FULL if mode == "full" else P.ASCC_VVVV_PACKED
    ints = P.ascc_build_ints(dev(B), dev(eps), o, precision=pc, vvvv_mode=vm)
    P.ascc_batch_reserve(ints, S)
    t1s = [dev(a[0]) for a in amps]
    t2s = [dev(a[1]) for a in amps]
    r1s = [torch.empty_like(t) for t in t1s]
    r2s = [torch.empty_like(t) for t in t2s]
    e = torch.empty(S, dtype=torch.float64, device="cuda")
    P.ascc_residual_batch(ints, t1s, t2s, r1s, r2s, e)
    torch.cuda.synchronize()
    eb = host(e)
    for k in range(S):
        r1, r2, ek = gpu_residual(P, ints, *amps[k])
        assert np.array_equal(host(r1s[k]), r1) and np.array_equal(host(r2s[k]), r2), f"state {k}"
        assert eb[k] == ek
        if prec == "fp64":
            ref1, ref2 = cs_ccsd.residual(B, np.diag(eps), *amps[k])
            assert max(np.abs(r1 - ref1).max(), np.abs(r2 - ref2).max()) <= 1e-10
    ints.close()


def test_batch_capacity_is_enforced(P):
    import torch

    from .gpu_util import dev

    B, eps = make_system(2, 3, 8, 1)
    ints = P.ascc_build_ints(dev(B), dev(eps), 2)
    P.ascc_batch_reserve(ints, 1)
    t1 = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    t2 = torch.zeros((2, 2, 3, 3), dtype=torch.float64, device="cuda")
    e = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(P.AsccError) as exc:
        P.ascc_residual_batch(ints, [t1, t1], [t2, t2], [t1.clone(), t1.clone()], [t2.clone(), t2.clone()], e)
    assert exc.value.code == P.ASCC_E_STATE
    ints.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("o,v,Q,S,G", [(3, 7, 15, 5, 2), (6, 40, 90, 5, 3), (9, 70, 130, 4, 4)])
def test_grouped_passes_equal_alone_bitwise(P, o, v, Q, S, G, prec):
    """Every term in batched passes of G states (each contraction one launch over the group against
    the shared integrals), from a caller workspace of exactly the reported size: each state's
    residual and energy equal the single-state ones bit for bit."""
    import torch

    from oracle import cs_ccsd

    from .gpu_util import dev, gpu_residual, host

    print(f"case o={o} v={v} Q={Q} S={S} G={G} prec={prec}", flush=True)
    B, eps = make_system(o, v, Q, 43, sigma=0.1)
    amps = [random_amplitudes(o, v, 400 + k, 0.05, 0.05) for k in range(S)]
    pc = {"fp64": P.ASCC_PREC_FP64, "fp32": P.ASCC_PREC_FP32, "bf16x3": P.ASCC_PREC_BF16X3}[prec]
    ints = P.ascc_build_ints(dev(B), dev(eps), o, precision=pc, vvvv_mode=P.ASCC_VVVV_PACKED)
    nbytes = P.ascc_batch_workspace_bytes(o, v, Q, S, G, precision=pc, vvvv_mode=P.ASCC_VVVV_PACKED)
    ws = torch.full((nbytes // 8,), float("nan"), dtype=torch.float64, device="cuda")
    P.ascc_batch_reserve_ws(ints, S, G, ws)
    T1 = dev(np.stack([a[0] for a in amps]))  # evenly spaced state arrays
    T2 = dev(np.stack([a[1] for a in amps]))
    R1, R2 = torch.empty_like(T1), torch.empty_like(T2)
    e = torch.empty(S, dtype=torch.float64, device="cuda")
    P.ascc_residual_batch(ints, list(T1), list(T2), list(R1), list(R2), e)
    torch.cuda.synchronize()
    eb = host(e)
    for k in range(S):
        r1, r2, ek = gpu_residual(P, ints, *amps[k])
        assert np.array_equal(host(R1[k]), r1) and np.array_equal(host(R2[k]), r2), f"state {k}"
        assert eb[k] == ek
        if prec == "fp64":
            ref1, ref2 = cs_ccsd.residual(B, np.diag(eps), *amps[k])
            assert max(np.abs(r1 - ref1).max(), np.abs(r2 - ref2).max()) <= 1e-10
    ints.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_sixteen_states_o30v270_grouped_equal_alone(P, prec):
    """The multi-state workload at its own size: 16 states of o30 v270 Q900 (packed vvvv), the other
    terms in passes of 3 states with a remainder pass, one ladder launch for all 16; every state's
    residual and energy equal its single-state ones bit for bit (the single-state path is the one
    pinned to the oracle at o20 v180 Q600)."""
    import torch

    from gen.synth_df import converging_sigma

    from .gpu_util import dev, host

    o, v, Q, S, G = 30, 270, 900, 16, 3
    print(f"case o={o} v={v} Q={Q} S={S} G={G} prec={prec}", flush=True)
    B, eps = make_system(o, v, Q, 44, sigma=converging_sigma(v, Q))
    pc = P.ASCC_PREC_FP64 if prec == "fp64" else P.ASCC_PREC_BF16X3
    ints = P.ascc_build_ints(dev(B), dev(eps), o, precision=pc, vvvv_mode=P.ASCC_VVVV_PACKED)
    del B
    nbytes = P.ascc_batch_workspace_bytes(o, v, Q, S, G, precision=pc, vvvv_mode=P.ASCC_VVVV_PACKED)
    ws = torch.empty((nbytes // 8,), dtype=torch.float64, device="cuda")
    P.ascc_batch_reserve_ws(ints, S, G, ws)
    gen = torch.Generator(device="cuda").manual_seed(45)
    T1 = 0.02 * torch.randn((S, o, v), dtype=torch.float64, device="cuda", generator=gen)
    T2 = 0.02 * torch.randn((S, o, o, v, v), dtype=torch.float64, device="cuda", generator=gen)
    T2 = 0.5 * (T2 + T2.permute(0, 2, 1, 4, 3))  # pair symmetry t_ij^ab = t_ji^ba
    R1, R2 = torch.empty_like(T1), torch.empty_like(T2)
    e = torch.empty(S, dtype=torch.float64, device="cuda")
    P.ascc_residual_batch(ints, list(T1), list(T2), list(R1), list(R2), e)
    torch.cuda.synchronize()
    eb = host(e)
    r1, r2 = torch.empty_like(T1[0]), torch.empty_like(T2[0])
    e1 = torch.empty(1, dtype=torch.float64, device="cuda")
    for k in range(S):
        P.ascc_residual(ints, T1[k], T2[k], r1, r2, e1)
        torch.cuda.synchronize()
        assert torch.equal(R1[k], r1) and torch.equal(R2[k], r2), f"state {k}"
        assert eb[k] == float(host(e1)[0]), f"state {k}"
    assert float(R2.abs().max()) > 1e-3
    ints.close()
    del T1, T2, R1, R2, ws, r1, r2
    torch.cuda.empty_cache()  # return the tens of GB held here to the device for the later tests
