"""ctypes declarations of libascc and torch-tensor marshalling (no arithmetic here)."""
from __future__ import annotations

import ctypes
import os
from pathlib import Path

import torch  # loaded first so that libascc binds to the HIP runtime torch already mapped

ASCC_OK = 0
ASCC_E_ARG = -1
ASCC_E_SHAPE = -2
ASCC_E_NOMEM = -3
ASCC_E_HIP = -4
ASCC_E_NONFINITE = -5
ASCC_E_NOT_CONVERGED = -6
ASCC_E_STATE = -7
ASCC_PREC_FP64 = 0
ASCC_PREC_FP32 = 1
ASCC_PREC_BF16X3 = 2
ASCC_VVVV_FULL = 0
ASCC_VVVV_PACKED = 1

_LIB = None


def library_path() -> Path:
    """The in-tree libascc.so (ASCC_LIB may name another build of the same sources)."""
    override = os.environ.get("ASCC_LIB")
    return Path(override) if override else Path(__file__).resolve().with_name("libascc.so")


class AsccError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libascc status {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("tol_rnorm", ctypes.c_double), ("tol_rmax", ctypes.c_double), ("tol_de", ctypes.c_double),
                ("maxiter", ctypes.c_int), ("diis_size", ctypes.c_int), ("diis_start", ctypes.c_int),
                ("level_shift", ctypes.c_double), ("lowp_rnorm", ctypes.c_double), ("lowp_maxiter", ctypes.c_int)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", ctypes.c_int), ("precision", ctypes.c_int),
                ("vvvv_mode", ctypes.c_int), ("use_graphs", ctypes.c_int), ("solve", Opts)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int), ("no", ctypes.c_int), ("nv", ctypes.c_int), ("naux", ctypes.c_int),
                ("status", ctypes.c_int), ("iterations", ctypes.c_int), ("lowp_iterations", ctypes.c_int),
                ("e_corr", ctypes.c_double), ("rnorm", ctypes.c_double), ("rmax", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("bytes", ctypes.c_size_t), ("e_ref", ctypes.c_double), ("hole", ctypes.c_int),
                ("particle", ctypes.c_int), ("bucket", ctypes.c_int), ("slot", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("e_corr", ctypes.c_double), ("rnorm", ctypes.c_double), ("rmax", ctypes.c_double),
                ("de", ctypes.c_double), ("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("lowp_iterations", ctypes.c_int), ("stalled", ctypes.c_int)]


class TwoAnsatzResult(ctypes.Structure):
    _fields_ = [("e_total", ctypes.c_double * 2), ("e_mean", ctypes.c_double), ("beta", ctypes.c_double * 2),
                ("solve", Result * 2), ("used", ctypes.c_int)]


EXPORTS = ("ascc_workspace_bytes", "ascc_build_ints", "ascc_residual", "ascc_diis_create", "ascc_diis_reset",
           "ascc_update", "ascc_solve", "ascc_ints_free", "ascc_diis_free", "ascc_ints_shape", "ascc_last_error",
           "ascc_phase_count", "ascc_phase_name", "ascc_timing_enable", "ascc_timing_read", "ascc_set_precision",
           "ascc_get_precision", "ascc_batch_reserve", "ascc_residual_batch", "ascc_build_ints_ws",
           "ascc_diis_create_ws", "ascc_server_create", "ascc_server_submit", "ascc_server_step",
           "ascc_server_info", "ascc_server_free", "ascc_build_ints_hbar", "ascc_initial_guess",
           "ascc_reference_energy", "ascc_set_plascc", "ascc_two_ansatz", "ascc_build_ints_hbar_ws",
           "ascc_server_submit_state", "ascc_plascc_workspace_bytes", "ascc_set_plascc_ws",
           "ascc_solve_noalloc", "ascc_batch_workspace_bytes", "ascc_batch_reserve_ws")


def load_library():
    """Load libascc.so once and declare every exported signature.  Raises if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not path.exists():
        raise RuntimeError(f"{path} is not built; run `python -m paper_2501_10515_amd.build` (no CPU fallback)")
    L = ctypes.CDLL(str(path))
    vp, c_int, c_double, c_size_p = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_size_t)
    L.ascc_workspace_bytes.argtypes = [c_int, c_int, c_int, c_int, c_int, c_int, c_size_p, c_size_p]
    L.ascc_build_ints.argtypes = [vp, vp, c_int, c_int, c_int, c_int, c_int, c_int, vp, ctypes.POINTER(vp)]
    L.ascc_residual.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.ascc_build_ints_hbar.argtypes = [vp, vp, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, vp,
                                       ctypes.POINTER(vp)]
    L.ascc_two_ansatz.argtypes = [vp, vp, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_double,
                                  ctypes.POINTER(Opts), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  ctypes.POINTER(TwoAnsatzResult), vp]
    L.ascc_initial_guess.argtypes = [vp, vp, c_int, c_int, c_int, c_int, c_double, c_double, vp]
    L.ascc_reference_energy.argtypes = [vp, ctypes.POINTER(c_double), vp]
    L.ascc_set_plascc.argtypes = [vp, c_int, c_int]
    L.ascc_plascc_workspace_bytes.argtypes = [c_int, c_int, c_int, c_size_p]
    L.ascc_set_plascc_ws.argtypes = [vp, c_int, c_int, vp, ctypes.c_size_t, vp]
    L.ascc_batch_workspace_bytes.argtypes = [c_int] * 7 + [c_size_p]
    L.ascc_batch_reserve_ws.argtypes = [vp, c_int, c_int, vp, ctypes.c_size_t]
    L.ascc_diis_create.argtypes = [vp, c_int, c_int, ctypes.POINTER(vp)]
    L.ascc_diis_reset.argtypes = [vp, vp]
    L.ascc_update.argtypes = [vp, vp, vp, vp, vp, vp, vp, c_double, vp, vp]
    L.ascc_solve.argtypes = [vp, ctypes.POINTER(Opts), vp, vp, ctypes.POINTER(Result), vp]
    L.ascc_solve_noalloc.argtypes = [vp, ctypes.POINTER(Opts), vp, vp, ctypes.POINTER(Result), vp]
    L.ascc_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    L.ascc_server_submit.argtypes = [vp, vp, vp, c_int, c_int, c_int, c_double, ctypes.POINTER(c_int)]
    L.ascc_server_submit_state.argtypes = [vp, vp, vp, c_int, c_int, c_int, c_int, c_int, c_int, c_double, c_int,
                                           c_double, ctypes.POINTER(c_int)]
    L.ascc_server_step.argtypes = [vp, c_double, ctypes.POINTER(c_int), ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    L.ascc_server_info.argtypes = [vp, c_int, ctypes.POINTER(RequestInfo)]
    L.ascc_server_free.argtypes = [vp]
    L.ascc_server_free.restype = None
    L.ascc_ints_free.argtypes = [vp]
    L.ascc_ints_free.restype = None
    L.ascc_diis_free.argtypes = [vp]
    L.ascc_diis_free.restype = None
    L.ascc_ints_shape.argtypes = [vp, ctypes.POINTER(c_int), ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    L.ascc_last_error.argtypes = []
    L.ascc_last_error.restype = ctypes.c_char_p
    L.ascc_phase_count.argtypes = []
    L.ascc_phase_name.argtypes = [c_int]
    L.ascc_phase_name.restype = ctypes.c_char_p
    L.ascc_timing_enable.argtypes = [vp, c_int]
    L.ascc_set_precision.argtypes = [vp, c_int]
    L.ascc_build_ints_ws.argtypes = [vp, vp, c_int, c_int, c_int, c_int, c_int, c_int, vp, ctypes.c_size_t, vp,
                                     ctypes.POINTER(vp)]
    L.ascc_build_ints_hbar_ws.argtypes = [vp, vp, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, vp,
                                          ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ascc_diis_create_ws.argtypes = [vp, c_int, c_int, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.ascc_batch_reserve.argtypes = [vp, c_int]
    L.ascc_residual_batch.argtypes = [vp, c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), vp, vp]
    L.ascc_get_precision.argtypes = [vp]
    L.ascc_timing_read.argtypes = [vp, ctypes.POINTER(c_double), ctypes.POINTER(c_int), c_int]
    for name in EXPORTS:
        if name not in ("ascc_ints_free", "ascc_diis_free", "ascc_last_error", "ascc_phase_name", "ascc_server_free"):
            getattr(L, name).restype = c_int
    _LIB = L
    return L


def ascc_last_error() -> str:
    return load_library().ascc_last_error().decode()


def _check(rc: int):
    if rc != ASCC_OK:
        raise AsccError(rc, ascc_last_error())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, name: str, shape=None) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def ascc_workspace_bytes(no: int, nv: int, naux: int, precision: int = ASCC_PREC_FP64,
                         vvvv_mode: int = ASCC_VVVV_FULL, diis_size: int = 8):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().ascc_workspace_bytes(no, nv, naux, precision, vvvv_mode, diis_size, ctypes.byref(a),
                                               ctypes.byref(b)))
    return a.value, b.value


class Ints:
    """Owner of an ascc_ints handle (frees it on close / garbage collection)."""

    def __init__(self, handle, no, nv, naux, workspace=None):
        self.handle = handle
        self.no, self.nv, self.naux = no, nv, naux
        self.workspace = workspace  # keeps a caller workspace alive as long as the handle

    def close(self):
        if self.handle:
            load_library().ascc_ints_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Diis:
    def __init__(self, handle, workspace=None):
        self.handle = handle
        self.workspace = workspace  # keeps a caller workspace alive as long as the handle

    def close(self):
        if self.handle:
            load_library().ascc_diis_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ascc_build_ints(B: torch.Tensor, fock: torch.Tensor, no: int, precision: int = ASCC_PREC_FP64,
                    vvvv_mode: int = ASCC_VVVV_FULL, stream=None) -> Ints:
    naux, n, n2 = B.shape
    if n != n2:
        raise ValueError("B must be [naux][n][n]")
    nv = n - no
    pB = _dev(B, "B")
    if fock.dim() == 1:
        pf, diag = _dev(fock, "fock", (n,)), 1
    else:
        pf, diag = _dev(fock, "fock", (n, n)), 0
    h = ctypes.c_void_p()
    _check(load_library().ascc_build_ints(pB, pf, diag, no, nv, naux, precision, vvvv_mode, _stream(stream),
                                          ctypes.byref(h)))
    return Ints(h, no, nv, naux)


def ascc_build_ints_hbar(B: torch.Tensor, fock: torch.Tensor, no: int, hole: int, particle: int,
                         precision: int = ASCC_PREC_FP64, vvvv_mode: int = ASCC_VVVV_FULL, stream=None,
                         s_sign: int = 1) -> Ints:
    """Integral set of the 1-CSF transformed Hamiltonian Hbar (``particle`` is a full orbital index;
    s_sign = -1: S of the hole-sign-flipped orbitals)."""
    naux, n, n2 = B.shape
    if n != n2:
        raise ValueError("B must be [naux][n][n]")
    nv = n - no
    pB = _dev(B, "B")
    if fock.dim() == 1:
        pf, diag = _dev(fock, "fock", (n,)), 1
    else:
        pf, diag = _dev(fock, "fock", (n, n)), 0
    h = ctypes.c_void_p()
    _check(load_library().ascc_build_ints_hbar(pB, pf, diag, no, nv, naux, precision, vvvv_mode, hole, particle,
                                               s_sign, _stream(stream), ctypes.byref(h)))
    return Ints(h, no, nv, naux)


def ascc_initial_guess(t1, t2, hole: int, particle: int, beta: float = 1.0, gamma: float = -0.5, stream=None):
    """Write T^P(0) = beta S + gamma S^2 into device t1 [no][nv] and t2 [no][no][nv][nv]."""
    no, nv = t1.shape
    _check(load_library().ascc_initial_guess(_dev(t1, "t1", (no, nv)), _dev(t2, "t2", (no, no, nv, nv)), no, nv,
                                             hole, particle, ctypes.c_double(beta), ctypes.c_double(gamma),
                                             _stream(stream)))


def ascc_build_ints_hbar_ws(B: torch.Tensor, fock: torch.Tensor, no: int, hole: int, particle: int,
                            workspace: torch.Tensor, precision: int = ASCC_PREC_FP64,
                            vvvv_mode: int = ASCC_VVVV_FULL, s_sign: int = 1, stream=None) -> Ints:
    """ascc_build_ints_hbar carved from a caller-owned device workspace (uint8 tensor)."""
    naux, n, n2 = B.shape
    if n != n2:
        raise ValueError("B must be [naux][n][n]")
    nv = n - no
    pB = _dev(B, "B")
    if fock.dim() == 1:
        pf, diag = _dev(fock, "fock", (n,)), 1
    else:
        pf, diag = _dev(fock, "fock", (n, n)), 0
    nbytes = workspace.numel() * workspace.element_size()
    h = ctypes.c_void_p()
    _check(load_library().ascc_build_ints_hbar_ws(pB, pf, diag, no, nv, naux, precision, vvvv_mode, hole, particle,
                                                  s_sign, _workspace_ptr(workspace, nbytes), nbytes, _stream(stream),
                                                  ctypes.byref(h)))
    return Ints(h, no, nv, naux, workspace)


def ascc_two_ansatz(B: torch.Tensor, fock: torch.Tensor, no: int, hole: int, particle: int, alpha: float, t1s, t2s,
                    precision: int = ASCC_PREC_FP64, vvvv_mode: int = ASCC_VVVV_FULL, tol_rnorm=1e-8, tol_rmax=0.0,
                    tol_de=0.0, maxiter=100, diis_size=8, diis_start=1, level_shift=0.0, lowp_rnorm=0.0,
                    lowp_maxiter=0, stream=None, raise_on_not_converged=True) -> dict:
    """Both ansatz of a 1-CSF state with Aufbau coefficient alpha; t1s, t2s: two device arrays each."""
    naux, n, n2 = B.shape
    if n != n2:
        raise ValueError("B must be [naux][n][n]")
    nv = n - no
    pB = _dev(B, "B")
    if fock.dim() == 1:
        pf, diag = _dev(fock, "fock", (n,)), 1
    else:
        pf, diag = _dev(fock, "fock", (n, n)), 0
    p1 = (ctypes.c_void_p * 2)(*[_dev(t, "t1", (no, nv)).value for t in t1s])
    p2 = (ctypes.c_void_p * 2)(*[_dev(t, "t2", (no, no, nv, nv)).value for t in t2s])
    opts = Opts(tol_rnorm, tol_rmax, tol_de, maxiter, diis_size, diis_start, level_shift, lowp_rnorm, lowp_maxiter)
    res = TwoAnsatzResult()
    rc = load_library().ascc_two_ansatz(pB, pf, diag, no, nv, naux, precision, vvvv_mode, hole, particle,
                                        ctypes.c_double(alpha), ctypes.byref(opts), p1, p2, ctypes.byref(res),
                                        _stream(stream))
    out = dict(e_total=[res.e_total[0], res.e_total[1]], e_mean=res.e_mean, beta=[res.beta[0], res.beta[1]],
               used=res.used,
               solves=[dict(e_corr=r.e_corr, rnorm=r.rnorm, iterations=r.iterations, converged=bool(r.converged),
                            lowp_iterations=r.lowp_iterations, stalled=bool(r.stalled)) for r in res.solve],
               status=rc)
    if rc != ASCC_OK and not (rc == ASCC_E_NOT_CONVERGED and not raise_on_not_converged):
        raise AsccError(rc, ascc_last_error())
    return out


def ascc_set_plascc(ints: Ints, hole: int, particle: int = -1):
    """Leave out the terms with two powers of the mixed doubles in later residuals (hole < 0: off)."""
    _check(load_library().ascc_set_plascc(ints.handle, hole, particle))


def ascc_plascc_workspace_bytes(no: int, nv: int, naux: int) -> int:
    """Exact device bytes of the PLASCC work buffers of an integral set of this shape."""
    b = ctypes.c_size_t()
    _check(load_library().ascc_plascc_workspace_bytes(no, nv, naux, ctypes.byref(b)))
    return b.value


def ascc_set_plascc_ws(ints: Ints, hole: int, particle: int, workspace, stream=None):
    """ascc_set_plascc with the work buffers carved from a caller workspace (a device tensor of at
    least ascc_plascc_workspace_bytes bytes that must outlive the handle); cleared on the stream."""
    nbytes = workspace.numel() * workspace.element_size()
    _check(load_library().ascc_set_plascc_ws(ints.handle, hole, particle, _dev(workspace, "workspace"), nbytes,
                                             _stream(stream)))
    ints._keep = getattr(ints, "_keep", []) + [workspace]


def ascc_reference_energy(ints: Ints, stream=None) -> float:
    """<phi_0|H|phi_0> of the integral set (of Hbar for an ascc_build_ints_hbar set); waits for the stream."""
    e0 = ctypes.c_double()
    _check(load_library().ascc_reference_energy(ints.handle, ctypes.byref(e0), _stream(stream)))
    return e0.value


def ascc_residual(ints: Ints, t1, t2, r1, r2, e, stream=None):
    o, v = ints.no, ints.nv
    _check(load_library().ascc_residual(ints.handle, _dev(t1, "t1", (o, v)), _dev(t2, "t2", (o, o, v, v)),
                                        _dev(r1, "r1", (o, v)), _dev(r2, "r2", (o, o, v, v)), _dev(e, "e", (1,)),
                                        _stream(stream)))


def ascc_diis_create(ints: Ints, max_vectors: int = 8, start: int = 1) -> Diis:
    h = ctypes.c_void_p()
    _check(load_library().ascc_diis_create(ints.handle, max_vectors, start, ctypes.byref(h)))
    return Diis(h)


def ascc_diis_reset(diis: Diis, stream=None):
    _check(load_library().ascc_diis_reset(diis.handle, _stream(stream)))


def ascc_update(ints: Ints, diis: Diis, t1, t2, r1, r2, e, stats, level_shift: float = 0.0, stream=None):
    o, v = ints.no, ints.nv
    _check(load_library().ascc_update(ints.handle, diis.handle, _dev(t1, "t1", (o, v)), _dev(t2, "t2", (o, o, v, v)),
                                      _dev(r1, "r1", (o, v)), _dev(r2, "r2", (o, o, v, v)), _dev(e, "e", (1,)),
                                      ctypes.c_double(level_shift), _dev(stats, "stats", (8,)), _stream(stream)))


def ascc_solve(ints: Ints, t1, t2, tol_rnorm=1e-8, tol_rmax=0.0, tol_de=0.0, maxiter=100, diis_size=8,
               diis_start=1, level_shift=0.0, lowp_rnorm=0.0, lowp_maxiter=0, stream=None,
               raise_on_not_converged=True, _entry="ascc_solve") -> dict:
    o, v = ints.no, ints.nv
    opts = Opts(tol_rnorm, tol_rmax, tol_de, maxiter, diis_size, diis_start, level_shift, lowp_rnorm, lowp_maxiter)
    res = Result()
    rc = getattr(load_library(), _entry)(ints.handle, ctypes.byref(opts), _dev(t1, "t1", (o, v)),
                                         _dev(t2, "t2", (o, o, v, v)), ctypes.byref(res), _stream(stream))
    out = dict(e_corr=res.e_corr, rnorm=res.rnorm, rmax=res.rmax, de=res.de, iterations=res.iterations,
               converged=bool(res.converged), lowp_iterations=res.lowp_iterations, stalled=bool(res.stalled),
               status=rc)
    if rc != ASCC_OK and not (rc == ASCC_E_NOT_CONVERGED and not raise_on_not_converged):
        raise AsccError(rc, ascc_last_error())
    return out


def ascc_solve_noalloc(ints: Ints, t1, t2, **kw) -> dict:
    """ascc_solve with the solver state in the library's fixed device array (no device allocation)."""
    return ascc_solve(ints, t1, t2, _entry="ascc_solve_noalloc", **kw)


def ascc_phase_count() -> int:
    return load_library().ascc_phase_count()


def ascc_phase_name(k: int) -> str:
    return load_library().ascc_phase_name(k).decode()


def ascc_timing_enable(ints: Ints, enable: bool = True):
    _check(load_library().ascc_timing_enable(ints.handle, 1 if enable else 0))


def ascc_timing_read(ints: Ints) -> dict:
    """{phase name: (total ms, intervals)} since the last read; waits for the recorded events."""
    n = ascc_phase_count()
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int * n)()
    _check(load_library().ascc_timing_read(ints.handle, ms, cnt, n))
    return {ascc_phase_name(k): (ms[k], cnt[k]) for k in range(n)}


def ascc_set_precision(ints: Ints, precision: int):
    _check(load_library().ascc_set_precision(ints.handle, precision))


def ascc_get_precision(ints: Ints) -> int:
    return load_library().ascc_get_precision(ints.handle)


def ascc_batch_reserve(ints: Ints, max_states: int):
    _check(load_library().ascc_batch_reserve(ints.handle, max_states))


def ascc_batch_workspace_bytes(no: int, nv: int, naux: int, max_states: int, group: int = 1,
                               precision: int = ASCC_PREC_FP64, vvvv_mode: int = ASCC_VVVV_FULL) -> int:
    b = ctypes.c_size_t()
    _check(load_library().ascc_batch_workspace_bytes(no, nv, naux, precision, vvvv_mode, max_states, group,
                                                     ctypes.byref(b)))
    return b.value


def ascc_batch_reserve_ws(ints: Ints, max_states: int, group: int = 1, workspace=None):
    """Batch capacity with `group` states per batched pass; workspace: a device tensor of at least
    ascc_batch_workspace_bytes bytes (kept alive with the handle), or None to let the library allocate."""
    if workspace is None:
        _check(load_library().ascc_batch_reserve_ws(ints.handle, max_states, group, None, 0))
        return
    nbytes = workspace.numel() * workspace.element_size()
    _check(load_library().ascc_batch_reserve_ws(ints.handle, max_states, group, _dev(workspace, "workspace"), nbytes))
    ints._keep = getattr(ints, "_keep", []) + [workspace]


def ascc_residual_batch(ints: Ints, t1s, t2s, r1s, r2s, e, stream=None):
    """Residuals of len(t1s) amplitude sets on one integral set; e is a device array [nstates]."""
    o, v = ints.no, ints.nv
    n = len(t1s)
    if not (len(t2s) == len(r1s) == len(r2s) == n):
        raise ValueError("t1s, t2s, r1s, r2s must have the same length")
    arr = ctypes.c_void_p * n
    p1 = arr(*[_dev(t, "t1", (o, v)) for t in t1s])
    p2 = arr(*[_dev(t, "t2", (o, o, v, v)) for t in t2s])
    q1 = arr(*[_dev(t, "r1", (o, v)) for t in r1s])
    q2 = arr(*[_dev(t, "r2", (o, o, v, v)) for t in r2s])
    _check(load_library().ascc_residual_batch(ints.handle, n, p1, p2, q1, q2, _dev(e, "e", (n,)), _stream(stream)))


def _workspace_ptr(ws: torch.Tensor, nbytes: int) -> ctypes.c_void_p:
    if ws.device.type != "cuda" or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous GPU tensor")
    if ws.numel() * ws.element_size() < nbytes:
        raise ValueError("workspace is smaller than required")
    if ws.data_ptr() % 256:
        raise ValueError("workspace must be 256-byte aligned")
    return ctypes.c_void_p(ws.data_ptr())


def ascc_build_ints_ws(B: torch.Tensor, fock: torch.Tensor, no: int, workspace: torch.Tensor,
                       precision: int = ASCC_PREC_FP64, vvvv_mode: int = ASCC_VVVV_FULL, stream=None) -> Ints:
    naux, n, _ = B.shape
    nv = n - no
    if fock.dim() == 1:
        pf, diag = _dev(fock, "fock", (n,)), 1
    else:
        pf, diag = _dev(fock, "fock", (n, n)), 0
    nbytes = workspace.numel() * workspace.element_size()
    h = ctypes.c_void_p()
    _check(load_library().ascc_build_ints_ws(_dev(B, "B"), pf, diag, no, nv, naux, precision, vvvv_mode,
                                             _workspace_ptr(workspace, 0), nbytes, _stream(stream), ctypes.byref(h)))
    return Ints(h, no, nv, naux, workspace)


def ascc_diis_create_ws(ints: Ints, workspace: torch.Tensor, max_vectors: int = 8, start: int = 1) -> Diis:
    nbytes = workspace.numel() * workspace.element_size()
    h = ctypes.c_void_p()
    _check(load_library().ascc_diis_create_ws(ints.handle, max_vectors, start, _workspace_ptr(workspace, 0), nbytes,
                                              ctypes.byref(h)))
    return Diis(h, workspace)


class Server:
    """Request server (ascc_server_*): submit host-side DF tensors, step the loop, read results."""

    def __init__(self, hbm_budget: int, max_active: int = 16, precision: int = ASCC_PREC_FP64,
                 vvvv_mode: int = ASCC_VVVV_PACKED, use_graphs: bool = True, tol_rnorm=1e-8, tol_rmax=0.0,
                 tol_de=0.0, maxiter=100, diis_size=8, diis_start=1, lowp_rnorm=0.0, lowp_maxiter=0):
        opts = ServerOpts(hbm_budget, max_active, precision, vvvv_mode, 1 if use_graphs else 0,
                          Opts(tol_rnorm, tol_rmax, tol_de, maxiter, diis_size, diis_start, 0.0, lowp_rnorm,
                               lowp_maxiter))
        h = ctypes.c_void_p()
        _check(load_library().ascc_server_create(ctypes.byref(opts), ctypes.byref(h)))
        self.handle = h

    def submit(self, B, eps, no: int, t_submit: float, hole: int = -1, particle: int = -1, s_sign: int = 1,
               beta: float = 1.0, plascc: bool = False) -> int:
        """Queue a ground-state request, or (hole >= 0) the 1-CSF ASCC state hole -> particle (PLASCC
        equations with plascc)."""
        import numpy as np

        B = np.ascontiguousarray(B, dtype=np.float64)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        naux, n, _ = B.shape
        rid = ctypes.c_int()
        pB, pe = B.ctypes.data_as(ctypes.c_void_p), eps.ctypes.data_as(ctypes.c_void_p)
        if hole < 0:
            _check(load_library().ascc_server_submit(self.handle, pB, pe, no, n - no, naux,
                                                     ctypes.c_double(t_submit), ctypes.byref(rid)))
        else:
            _check(load_library().ascc_server_submit_state(self.handle, pB, pe, no, n - no, naux, hole, particle,
                                                           s_sign, ctypes.c_double(beta), 1 if plascc else 0,
                                                           ctypes.c_double(t_submit), ctypes.byref(rid)))
        return rid.value

    def step(self, now: float):
        q, r, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load_library().ascc_server_step(self.handle, ctypes.c_double(now), ctypes.byref(q), ctypes.byref(r),
                                               ctypes.byref(d)))
        return q.value, r.value, d.value

    def info(self, rid: int) -> dict:
        x = RequestInfo()
        _check(load_library().ascc_server_info(self.handle, rid, ctypes.byref(x)))
        return {k: getattr(x, k) for k, _ in RequestInfo._fields_}

    def close(self):
        if self.handle:
            load_library().ascc_server_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
