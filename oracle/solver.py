"""Diagonal approximate-Jacobian amplitude update with DIIS, and the convergence test, FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper Sec. III.B: the amplitudes are updated with the diagonal approximate Jacobian, i.e. the
orbital-energy denominators, and the iteration is accelerated with DIIS; Sec. III.A: the
paper's own convergence test is max|R| <= 1e-5 and |dE| < 1e-7 Eh per iteration.

The paper leaves the DIIS details to earlier work; this module takes the common reading:

* Jacobi step: t <- t + R / D with D_i^a = e_i - e_a and D_ij^ab = e_i + e_j - e_a - e_b
  (optionally D - shift, a level shift, which leaves the fixed point unchanged);
* DIIS error vector: the Jacobi step itself, Delta = R / D, over t1 (+) t2 (full closed-shell
  arrays, plain dot product); the extrapolated quantity is the post-step amplitude vector;
* up to ``diis_size`` (default 8) pairs are kept, oldest dropped first; pairs are stored from
  0-based iteration ``diis_start`` (default 1, i.e. the second iteration) and extrapolation
  starts once two pairs are stored;
* the bordered system [[B, -1], [-1, 0]] [c; lam] = [0; -1], B_kl = <e_k, e_l>, is solved by
  Gaussian elimination with partial pivoting; if a pivot falls below 1e-14 * max|B| the oldest
  pair is dropped and the solve retried.
"""
from __future__ import annotations

import numpy as np


def denominators(eps: np.ndarray, no: int, shift: float = 0.0):
    e_o, e_v = eps[:no], eps[no:]
    d1 = e_o[:, None] - e_v[None, :] - shift
    d2 = e_o[:, None, None, None] + e_o[None, :, None, None] - e_v[None, None, :, None] - e_v[None, None, None, :] - shift
    return d1, d2


def solve_bordered(Bm: np.ndarray, rel_pivot: float = 1e-14):
    """Gaussian elimination with partial pivoting on the DIIS bordered system; None if ill-conditioned."""
    m = Bm.shape[0]
    A = np.zeros((m + 1, m + 2))
    A[:m, :m] = Bm
    A[:m, m] = -1.0
    A[m, :m] = -1.0
    A[m, m + 1] = -1.0
    scale = np.abs(Bm).max()
    for col in range(m + 1):
        piv = col + int(np.argmax(np.abs(A[col:, col])))
        if abs(A[piv, col]) < rel_pivot * scale:
            return None
        if piv != col:
            A[[col, piv]] = A[[piv, col]]
        for r in range(col + 1, m + 1):
            A[r] -= (A[r, col] / A[col, col]) * A[col]
    x = np.zeros(m + 1)
    for r in range(m, -1, -1):
        x[r] = (A[r, m + 1] - A[r, r + 1:m + 1] @ x[r + 1:]) / A[r, r]
    return x[:m]


class DIIS:
    def __init__(self, size: int = 8):
        self.size = size
        self.vecs: list = []
        self.errs: list = []

    def push(self, vec: np.ndarray, err: np.ndarray):
        self.vecs.append(vec.copy())
        self.errs.append(err.copy())
        while len(self.vecs) > self.size:
            self.vecs.pop(0)
            self.errs.pop(0)

    def extrapolate(self):
        while len(self.vecs) >= 2:
            m = len(self.vecs)
            Bm = np.array([[self.errs[k] @ self.errs[l] for l in range(m)] for k in range(m)])
            c = solve_bordered(Bm)
            if c is not None:
                return sum(ck * vk for ck, vk in zip(c, self.vecs)), c
            self.vecs.pop(0)
            self.errs.pop(0)
        return None, None


def solve(residual_fn, energy_fn, eps, t1, t2, maxiter=100, tol_rnorm=1e-8, tol_rmax=None, tol_de=None,
          diis_size=8, diis_start=1, shift=0.0, callback=None):
    """Iterate t <- DIIS(t + R/D) from (t1, t2) until the requested tests pass.

    ``residual_fn(t1, t2) -> (r1, r2)`` and ``energy_fn(t1, t2) -> E`` evaluate at the same t.
    Convergence (checked on the residual of the current t, before any update): every given
    tolerance holds, with rnorm = sqrt(|r1|^2 + |r2|^2), rmax = max|R| and dE the change of E
    since the previous iteration.  Returns a dict with the final amplitudes, energy, history.
    """
    no, nv = t1.shape
    d1, d2 = denominators(eps, no, shift)
    n1 = t1.size
    diis = DIIS(diis_size)
    t1, t2 = t1.copy(), t2.copy()
    e_prev = None
    hist = []
    converged = False
    for it in range(maxiter):
        r1, r2 = residual_fn(t1, t2)
        e = energy_fn(t1, t2)
        rnorm = float(np.sqrt(np.sum(r1 * r1) + np.sum(r2 * r2)))
        rmax = float(max(np.abs(r1).max(), np.abs(r2).max()))
        de = float("inf") if e_prev is None else e - e_prev
        hist.append(dict(it=it, E=e, dE=de, rnorm=rnorm, rmax=rmax, ndiis=len(diis.vecs)))
        if callback is not None:
            callback(hist[-1])
        if not (np.isfinite(rnorm) and np.isfinite(e)):
            break
        ok = (tol_rnorm is None or rnorm <= tol_rnorm) and (tol_rmax is None or rmax <= tol_rmax) and \
             (tol_de is None or abs(de) < tol_de)
        if ok:
            converged = True
            break
        e_prev = e
        s1, s2 = r1 / d1, r2 / d2
        t1 = t1 + s1
        t2 = t2 + s2
        if it >= diis_start:
            diis.push(np.concatenate([t1.ravel(), t2.ravel()]), np.concatenate([s1.ravel(), s2.ravel()]))
            x, _ = diis.extrapolate()
            if x is not None:
                t1 = x[:n1].reshape(no, nv)
                t2 = x[n1:].reshape(no, no, nv, nv)
    return dict(t1=t1, t2=t2, E=hist[-1]["E"], converged=converged, iterations=len(hist), history=hist)
