"""Drive the whole libascc launch sequence without a GPU (ASCC_DRY_RUN=1) and report.

Run as a separate process (the library reads ASCC_DRY_RUN once).  Caller buffers are fake,
unbacked addresses; the library registers them with the sizes the C ABI defines and checks
the lowest and highest element of every GEMM, permute, copy and kernel launch against them.
Prints one line "OK <no> <nv> <naux>" per shape, or the failing status and message.
"""
import ctypes
import os
import sys

os.environ["ASCC_DRY_RUN"] = "1"
from pathlib import Path  # noqa: E402

LIB = Path(__file__).resolve().parents[1] / "paper_2501_10515_amd" / "libascc.so"


class Opts(ctypes.Structure):
    _fields_ = [("tol_rnorm", ctypes.c_double), ("tol_rmax", ctypes.c_double), ("tol_de", ctypes.c_double),
                ("maxiter", ctypes.c_int), ("diis_size", ctypes.c_int), ("diis_start", ctypes.c_int),
                ("level_shift", ctypes.c_double), ("lowp_rnorm", ctypes.c_double), ("lowp_maxiter", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("e_corr", ctypes.c_double), ("rnorm", ctypes.c_double), ("rmax", ctypes.c_double),
                ("de", ctypes.c_double), ("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("lowp_iterations", ctypes.c_int), ("stalled", ctypes.c_int)]


class TwoAnsatzResult(ctypes.Structure):
    _fields_ = [("e_total", ctypes.c_double * 2), ("e_mean", ctypes.c_double), ("beta", ctypes.c_double * 2),
                ("solve", Result * 2), ("used", ctypes.c_int)]


def main(shapes):
    L = ctypes.CDLL(str(LIB))
    vp = ctypes.c_void_p
    L.ascc_last_error.restype = ctypes.c_char_p
    L.ascc_build_ints.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.ascc_residual.argtypes = [vp] * 7
    L.ascc_diis_create.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    L.ascc_update.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, vp, vp]
    L.ascc_solve.argtypes = [vp, ctypes.POINTER(Opts), vp, vp, ctypes.POINTER(Result), vp]
    L.ascc_solve_noalloc.argtypes = [vp, ctypes.POINTER(Opts), vp, vp, ctypes.POINTER(Result), vp]
    L.ascc_batch_reserve.argtypes = [vp, ctypes.c_int]
    L.ascc_batch_reserve_ws.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t]
    L.ascc_batch_workspace_bytes.argtypes = [ctypes.c_int] * 7 + [ctypes.POINTER(ctypes.c_size_t)]
    L.ascc_residual_batch.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), vp, vp]
    L.ascc_workspace_bytes.argtypes = [ctypes.c_int] * 6 + [ctypes.POINTER(ctypes.c_size_t)] * 2
    L.ascc_build_ints_ws.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ascc_diis_create_ws.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.ascc_ints_free.argtypes = [vp]
    L.ascc_diis_free.argtypes = [vp]
    L.ascc_build_ints_hbar.argtypes = [vp, vp] + [ctypes.c_int] * 9 + [vp, ctypes.POINTER(vp)]
    L.ascc_initial_guess.argtypes = [vp, vp] + [ctypes.c_int] * 4 + [ctypes.c_double] * 2 + [vp]
    L.ascc_reference_energy.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
    L.ascc_set_plascc.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.ascc_plascc_workspace_bytes.argtypes = [ctypes.c_int] * 3 + [ctypes.POINTER(ctypes.c_size_t)]
    L.ascc_set_plascc_ws.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp]
    L.ascc_build_ints_hbar_ws.argtypes = [vp, vp] + [ctypes.c_int] * 9 + [vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ascc_two_ansatz.argtypes = [vp, vp] + [ctypes.c_int] * 8 + [ctypes.c_double, ctypes.POINTER(Opts),
                                                                    ctypes.POINTER(vp), ctypes.POINTER(vp),
                                                                    ctypes.POINTER(TwoAnsatzResult), vp]
    ok = True
    for shape in shapes:
        o, v, Q, diag = shape[:4]
        mode = shape[4] if len(shape) > 4 else 0
        prec = shape[5] if len(shape) > 5 else 0
        n = o + v
        base = [0x200000000000]

        def fake(nbytes):  # distinct, page-aligned, never dereferenced
            p = base[0]
            base[0] += (nbytes + 2 * 4096) // 4096 * 4096
            return vp(p)

        B = fake(8 * Q * n * n)
        F = fake(8 * (n if diag else n * n))
        h = vp()
        rc = L.ascc_build_ints(B, F, diag, o, v, Q, prec, mode, None, ctypes.byref(h))
        msgs = []
        if rc == 0:
            t1, t2, r1, r2, e, st = (fake(8 * o * v), fake(8 * o * o * v * v), fake(8 * o * v),
                                     fake(8 * o * o * v * v), fake(8), fake(64))
            rc = L.ascc_residual(h, t1, t2, r1, r2, e, None)
            if rc == 0:
                d = vp()
                rc = L.ascc_diis_create(h, 8, 1, ctypes.byref(d))
                for _ in range(3):
                    if rc == 0:
                        rc = L.ascc_update(h, d, t1, t2, r1, r2, e, ctypes.c_double(0.0), st, None)
                L.ascc_diis_free(d)
            if rc == 0:  # a batch of three states
                S = 3
                rc = L.ascc_batch_reserve(h, S)
                arr = vp * S
                bt1 = arr(*[fake(8 * o * v) for _ in range(S)])
                bt2 = arr(*[fake(8 * o * o * v * v) for _ in range(S)])
                br1 = arr(*[fake(8 * o * v) for _ in range(S)])
                br2 = arr(*[fake(8 * o * o * v * v) for _ in range(S)])
                if rc == 0:
                    rc = L.ascc_residual_batch(h, S, bt1, bt2, br1, br2, fake(8 * S), None)
                if rc == 0:  # five evenly spaced states in batched passes of two, from an exact workspace
                    S5, G = 5, 2
                    wb = ctypes.c_size_t()
                    rc = L.ascc_batch_workspace_bytes(o, v, Q, prec, mode, S5, G, ctypes.byref(wb))
                    if rc == 0:
                        rc = L.ascc_batch_reserve_ws(h, S5, G, fake(wb.value), wb.value)
                    arr5 = vp * S5
                    st1, st2, sr1, sr2 = (fake(8 * o * v * S5), fake(8 * o * o * v * v * S5), fake(8 * o * v * S5),
                                          fake(8 * o * o * v * v * S5))
                    bt1 = arr5(*[st1.value + 8 * o * v * k for k in range(S5)])
                    bt2 = arr5(*[st2.value + 8 * o * o * v * v * k for k in range(S5)])
                    br1 = arr5(*[sr1.value + 8 * o * v * k for k in range(S5)])
                    br2 = arr5(*[sr2.value + 8 * o * o * v * v * k for k in range(S5)])
                    if rc == 0:
                        rc = L.ascc_residual_batch(h, S5, bt1, bt2, br1, br2, fake(8 * S5), None)
            if rc == 0:
                res = Result()
                rc = L.ascc_solve(h, ctypes.byref(Opts(1e-8, 0, 0, 3, 8, 1, 0.0, 1e-3, 1)), t1, t2, ctypes.byref(res),
                                  None)
            if rc == 0:  # the same solve in the fixed solver array: it fits up to about o8 v72 with m = 8
                res = Result()
                rcn = L.ascc_solve_noalloc(h, ctypes.byref(Opts(1e-8, 0, 0, 3, 8, 1, 0.0, 1e-3, 1)), t1, t2,
                                           ctypes.byref(res), None)
                fits = 18 * (o * v + o * o * v * v) * 8 + (1 << 20) <= 64 << 20
                if (rcn == 0) != fits or (rcn != 0 and rcn != -3):
                    rc = -102
                    print(f"ascc_solve_noalloc status {rcn} (fits {fits})", flush=True)
            L.ascc_ints_free(h)
        if rc == 0:  # the transformed Hamiltonian of a 1-CSF state, its guess and one residual
            h4 = vp()
            rc = L.ascc_build_ints_hbar(B, F, diag, o, v, Q, prec, mode, o - 1, o, -1, None, ctypes.byref(h4))
            if rc == 0:
                t1, t2, r1, r2, e = (fake(8 * o * v), fake(8 * o * o * v * v), fake(8 * o * v),
                                     fake(8 * o * o * v * v), fake(8))
                rc = L.ascc_initial_guess(t1, t2, o, v, o - 1, o, ctypes.c_double(1.0), ctypes.c_double(-0.5), None)
                if rc == 0:
                    rc = L.ascc_residual(h4, t1, t2, r1, r2, e, None)
                if rc == 0:  # and with the partial linearisation of the same primaries
                    rc = L.ascc_set_plascc(h4, o - 1, o)
                if rc == 0:
                    rc = L.ascc_residual(h4, t1, t2, r1, r2, e, None)
                if rc == 0:
                    rc = L.ascc_set_plascc(h4, 0, o + v - 1)
                if rc == 0:
                    rc = L.ascc_residual(h4, t1, t2, r1, r2, e, None)
                if rc == 0:
                    e0 = ctypes.c_double(1.0)
                    rc = L.ascc_reference_energy(h4, ctypes.byref(e0), None)
                L.ascc_ints_free(h4)
            if rc == 0:  # the state's integral set carved from an exact-size workspace
                ib, dbytes = ctypes.c_size_t(), ctypes.c_size_t()
                rc = L.ascc_workspace_bytes(o, v, Q, prec, mode, 8, ctypes.byref(ib), ctypes.byref(dbytes))
                h5 = vp()
                if rc == 0:
                    rc = L.ascc_build_ints_hbar_ws(B, F, diag, o, v, Q, prec, mode, 0, o + v - 1, 1, fake(ib.value),
                                                   ib.value, None, ctypes.byref(h5))
                if rc == 0:
                    t1, t2, r1, r2, e = (fake(8 * o * v), fake(8 * o * o * v * v), fake(8 * o * v),
                                         fake(8 * o * o * v * v), fake(8))
                    rc = L.ascc_residual(h5, t1, t2, r1, r2, e, None)
                    if rc == 0:  # PLASCC buffers carved from an exact-size workspace (one byte less refused)
                        pb = ctypes.c_size_t()
                        rc = L.ascc_plascc_workspace_bytes(o, v, Q, ctypes.byref(pb))
                        if rc == 0 and L.ascc_set_plascc_ws(h5, 0, o + v - 1, fake(pb.value), pb.value - 1, None) != -3:
                            rc = -101
                            print("undersized PLASCC workspace accepted", flush=True)
                        if rc == 0:
                            rc = L.ascc_set_plascc_ws(h5, 0, o + v - 1, fake(pb.value), pb.value, None)
                        if rc == 0:
                            rc = L.ascc_residual(h5, t1, t2, r1, r2, e, None)
                    L.ascc_ints_free(h5)
            if rc == 0:  # both ansatz of the state, each built, solved and freed in turn
                t1s = (vp * 2)(fake(8 * o * v), fake(8 * o * v))
                t2s = (vp * 2)(fake(8 * o * o * v * v), fake(8 * o * o * v * v))
                tres = TwoAnsatzResult()
                rc = L.ascc_two_ansatz(B, F, diag, o, v, Q, prec, mode, o - 1, o, 0.1,
                                       ctypes.byref(Opts(1e-8, 0, 0, 3, 8, 1, 0.0, 1e-3, 1)), t1s, t2s,
                                       ctypes.byref(tres), None)
        if rc == 0:  # the same build and an update carved from exact-size workspaces
            ib, dbytes = ctypes.c_size_t(), ctypes.c_size_t()
            rc = L.ascc_workspace_bytes(o, v, Q, prec, mode, 8, ctypes.byref(ib), ctypes.byref(dbytes))
            h2 = vp()
            if rc == 0:
                rc = L.ascc_build_ints_ws(B, F, diag, o, v, Q, prec, mode, fake(ib.value), ib.value, None,
                                          ctypes.byref(h2))
            if rc == 0:
                d2 = vp()
                rc = L.ascc_diis_create_ws(h2, 8, 1, fake(dbytes.value), dbytes.value, ctypes.byref(d2))
                t1, t2, r1, r2, e, st = (fake(8 * o * v), fake(8 * o * o * v * v), fake(8 * o * v),
                                         fake(8 * o * o * v * v), fake(8), fake(64))
                if rc == 0:
                    rc = L.ascc_residual(h2, t1, t2, r1, r2, e, None)
                if rc == 0:
                    rc = L.ascc_update(h2, d2, t1, t2, r1, r2, e, ctypes.c_double(0.0), st, None)
                L.ascc_diis_free(d2)
            if rc == 0:  # one byte short of the reported size must be refused
                h3 = vp()
                rc3 = L.ascc_build_ints_ws(B, F, diag, o, v, Q, prec, mode, fake(ib.value), ib.value - 1, None,
                                           ctypes.byref(h3))
                if rc3 != -3:
                    rc = -100
                    print("undersized workspace accepted", flush=True)
            L.ascc_ints_free(h2)
        if rc == 0:
            print(f"OK {o} {v} {Q} mode {mode} prec {prec}", flush=True)
        else:
            ok = False
            print(f"FAIL {o} {v} {Q} mode {mode} status {rc}: {L.ascc_last_error().decode()}", flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    shapes = [tuple(int(x) for x in s.split(",")) for s in sys.argv[1:]]
    sys.exit(main(shapes))
