"""Error paths of the C ABI forced from the host: a non-finite amplitude, a request larger than the
server's HBM budget, and a solve that reaches maxiter.  Every kernel runs normally; only the values
or the sizes passed in are out of range."""
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


def test_nan_amplitude_sets_the_nonfinite_flag_and_fails_the_solve(P):
    import torch

    o, v, Q = 4, 16, 48
    B, eps = make_system(o, v, Q, 3, sigma=converging_sigma(v, Q))
    ints = P.ascc_build_ints(torch.from_numpy(B).cuda(), torch.from_numpy(eps).cuda(), o)
    t1 = torch.zeros((o, v), dtype=torch.float64, device="cuda")
    t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    t2[1, 2, 3, 4] = float("nan")
    t2[2, 1, 4, 3] = float("nan")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    e = torch.empty(1, dtype=torch.float64, device="cuda")
    stats = torch.empty(8, dtype=torch.float64, device="cuda")
    diis = P.ascc_diis_create(ints, 8, 1)
    P.ascc_residual(ints, t1, t2, r1, r2, e)
    P.ascc_update(ints, diis, t1, t2, r1, r2, e, stats)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    diis.close()
    assert int(st[5]) & 1, st
    t2[1, 2, 3, 4] = float("nan")
    t2[2, 1, 4, 3] = float("nan")
    with pytest.raises(P.AsccError) as exc:
        P.ascc_solve(ints, t1, t2, tol_rnorm=1e-8, maxiter=20)
    ints.close()
    assert exc.value.code == P.ASCC_E_NONFINITE and "non-finite" in str(exc.value)


def test_maxiter_returns_not_converged_with_the_evaluated_amplitudes(P):
    """An unconverged solve reports the statistics of the amplitudes it returns."""
    import torch

    from .gpu_util import gpu_residual

    o, v, Q = 5, 20, 60
    B, eps = make_system(o, v, Q, 0, sigma=converging_sigma(v, Q))
    ints = P.ascc_build_ints(torch.from_numpy(B).cuda(), torch.from_numpy(eps).cuda(), o)
    t1 = torch.zeros((o, v), dtype=torch.float64, device="cuda")
    t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    res = P.ascc_solve(ints, t1, t2, tol_rnorm=1e-12, maxiter=4, raise_on_not_converged=False)
    assert res["status"] == P.ASCC_E_NOT_CONVERGED and not res["converged"] and res["iterations"] == 4
    with pytest.raises(P.AsccError) as exc:
        P.ascc_solve(ints, torch.zeros_like(t1), torch.zeros_like(t2), tol_rnorm=1e-12, maxiter=4)
    assert exc.value.code == P.ASCC_E_NOT_CONVERGED
    r1, r2, e = gpu_residual(P, ints, t1.cpu().numpy(), t2.cpu().numpy())
    ints.close()
    rnorm = float(np.sqrt((r1 ** 2).sum() + (r2 ** 2).sum()))
    print(res, e, rnorm, flush=True)
    assert e == res["e_corr"]
    assert abs(rnorm - res["rnorm"]) <= 1e-12 * rnorm
    assert max(np.abs(r1).max(), np.abs(r2).max()) == res["rmax"]
    assert res["rnorm"] > 1e-8  # really unconverged after four iterations


def test_request_larger_than_the_budget_is_refused_at_submit(P):
    """ASCC_E_NOMEM at submit for a request whose footprint exceeds the whole budget; the requests
    that fit are served to convergence."""
    small = []
    for k, o in enumerate([3, 4]):
        v, Q = 4 * o, 15 * o
        B, eps = make_system(o, v, Q, 600 + k, sigma=converging_sigma(v, Q))
        small.append((o, B, eps))
    need = [sum(P.ascc_workspace_bytes(o, B.shape[1] - o, B.shape[0], P.ASCC_PREC_FP64, P.ASCC_VVVV_PACKED, 8))
            for o, B, _ in small]
    budget = 3 * max(need)
    ob, vb = 12, 96
    big_need = sum(P.ascc_workspace_bytes(ob, vb, 3 * (ob + vb), P.ASCC_PREC_FP64, P.ASCC_VVVV_PACKED, 8))
    assert big_need > budget
    Bb, eb = make_system(ob, vb, 3 * (ob + vb), 7, sigma=converging_sigma(vb, 3 * (ob + vb)))
    srv = P.Server(budget, max_active=4, precision=P.ASCC_PREC_FP64, vvvv_mode=P.ASCC_VVVV_PACKED, tol_rnorm=1e-8,
                   maxiter=200)
    t0 = time.perf_counter()
    ids = [srv.submit(small[0][1], small[0][2], small[0][0], 0.0)]
    with pytest.raises(P.AsccError) as exc:
        srv.submit(Bb, eb, ob, 0.0)
    assert exc.value.code == P.ASCC_E_NOMEM
    ids.append(srv.submit(small[1][1], small[1][2], small[1][0], 0.0))
    while True:
        q, r, d = srv.step(time.perf_counter() - t0)
        if d == len(ids):
            break
        assert time.perf_counter() - t0 < 60, "server did not finish"
    infos = [srv.info(i) for i in ids]
    srv.close()
    assert all(x["status"] == 0 for x in infos)


CHECK_MODE_CHILD = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import paper_2501_10515_amd as P
from gen.synth_df import make_system
P.load_library()
o, v, Q = 3, 7, 15
B, eps = make_system(o, v, Q, 5)
dB = torch.from_numpy(B).cuda()
P.ascc_build_ints(dB, torch.from_numpy(eps).cuda(), o).close()
print("ordered ok", flush=True)
fock = np.diag(eps) + 0.01 * np.ones((o + v, o + v))
P.ascc_build_ints(dB, torch.from_numpy(fock).cuda(), o).close()
print("full ordered ok", flush=True)
for name, f in (("diag", eps.copy()), ("full", np.diag(eps))):
    k = o - 1
    val = eps[o] + 0.1  # the last occupied energy above the first virtual one
    if f.ndim == 1:
        f[k] = val
    else:
        f[k, k] = val
    try:
        P.ascc_build_ints(dB, torch.from_numpy(f).cuda(), o).close()
        print(name, "no error", flush=True)
    except P.AsccError as exc:
        print(name, "code", exc.code, flush=True)
"""


def test_check_mode_refuses_crossed_orbital_energies(P, tmp_path):
    """With ASCC_CHECK_BOUNDS=1 (read once per process, so in a child) an integral build whose
    largest occupied orbital energy is not below the smallest virtual one fails with ASCC_E_ARG,
    for a diagonal and for a full Fock matrix; ordered energies build as before."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = tmp_path / "check_mode_child.py"
    script.write_text(CHECK_MODE_CHILD)
    print("case: check-mode child, o3 v7 Q15", flush=True)
    r = subprocess.run([sys.executable, str(script), root], capture_output=True, text=True, timeout=240,
                       env=dict(os.environ, ASCC_CHECK_BOUNDS="1"), cwd=root)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = r.stdout.split("\n")
    assert "ordered ok" in lines and "full ordered ok" in lines, r.stdout
    assert f"diag code {P.ASCC_E_ARG}" in lines and f"full code {P.ASCC_E_ARG}" in lines, r.stdout
