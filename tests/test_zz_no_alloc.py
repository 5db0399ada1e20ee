"""ascc_solve_noalloc (the solve whose solver state lives in the library's fixed device array)
against ascc_solve, through the C ABI: the same amplitudes, energy and statistics bit for bit, on two
calls in a row (the second on a smaller system, over the first call's leftover contents), and a
clear refusal of a solver state larger than the array."""
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


def _pair(P, o, v, Q, seed, precision, **kw):
    import torch

    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    ints = P.ascc_build_ints(torch.from_numpy(B).cuda(), torch.from_numpy(eps).cuda(), o, precision=precision,
                             vvvv_mode=P.ASCC_VVVV_PACKED)
    out = []
    for solve in (P.ascc_solve, P.ascc_solve_noalloc):
        t1 = torch.zeros((o, v), dtype=torch.float64, device="cuda")
        t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
        r = solve(ints, t1, t2, **kw)
        out.append((r, t1.cpu().numpy(), t2.cpu().numpy()))
    ints.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_noalloc_solve_equals_solve_on_two_calls(P, precision):
    pc = P.ASCC_PREC_FP64 if precision == "fp64" else P.ASCC_PREC_BF16X3
    kw = dict(tol_rnorm=1e-9, maxiter=100, lowp_rnorm=1e-6 if precision != "fp64" else 0.0)
    for o, v, Q, seed in [(6, 30, 90, 21), (4, 16, 60, 22)]:  # the second call is smaller
        print(f"case o={o} v={v} Q={Q} {precision}", flush=True)
        (ra, t1a, t2a), (rb, t1b, t2b) = _pair(P, o, v, Q, seed, pc, **kw)
        print(ra, rb, flush=True)
        assert ra["converged"] and rb["converged"]
        assert ra == rb  # every statistic, bit for bit
        assert np.array_equal(t1a, t1b) and np.array_equal(t2a, t2b)


def test_noalloc_solve_refuses_a_state_beyond_its_array(P):
    import torch

    o, v, Q = 10, 90, 300  # (2*8 + 2)(ov + o^2 v^2) doubles = 117 MB > 64 MiB
    B, eps = make_system(o, v, Q, 23, sigma=converging_sigma(v, Q))
    ints = P.ascc_build_ints(torch.from_numpy(B).cuda(), torch.from_numpy(eps).cuda(), o,
                             vvvv_mode=P.ASCC_VVVV_PACKED)
    t1 = torch.zeros((o, v), dtype=torch.float64, device="cuda")
    t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    with pytest.raises(P.AsccError) as exc:
        P.ascc_solve_noalloc(ints, t1, t2, tol_rnorm=1e-8, maxiter=5)
    assert exc.value.code == P.ASCC_E_NOMEM and "bytes" in str(exc.value)
    # a smaller DIIS history fits the same system? (2*2 + 2) * 810900 * 8 = 38.9 MB: yes
    r = P.ascc_solve_noalloc(ints, t1, t2, tol_rnorm=1e-8, maxiter=200, diis_size=2)
    ints.close()
    assert r["converged"]
