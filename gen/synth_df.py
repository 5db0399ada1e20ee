"""Seeded synthetic density-fitted integrals, orbital energies and amplitudes.

Recipe (stated once, used by every consumer):

* ``B`` has shape ``(naux, n, n)`` with ``n = no + nv``, occupied orbitals first.
  It is drawn i.i.d. N(0, sigma^2) in C order from ``numpy.random.default_rng(seed)``,
  then the strict upper triangle of every ``B[Q]`` is mirrored onto the lower one,
  so ``B[Q, p, q] == B[Q, q, p]`` and every entry keeps the N(0, sigma^2) marginal.
  The two-electron integrals are then ``(pq|rs) = sum_Q B[Q,p,q] B[Q,r,s]``.
* After ``B``, the same generator draws the occupied orbital energies
  ``sort(uniform(-2.0, -0.3, no))`` and then the virtual ones ``sort(uniform(0.1, 5.0, nv))``.
  The Fock matrix is ``diag(eps)``.
* ``sigma`` defaults to 0.05.  ``converging_sigma`` gives the rescaled width used by the
  "convergence variant" (same shapes and seeds, ``naux * nv * sigma^2`` held at its
  no=5, nv=20, naux=60 value of 3.0 Eh).

Nothing in this module computes a coupled-cluster quantity.
"""
from __future__ import annotations

import numpy as np

SIGMA = 0.05


def converging_sigma(nv: int, naux: int) -> float:
    """Width that keeps naux*nv*sigma^2 = 1200*0.05^2 (the small-case value)."""
    return SIGMA * float(np.sqrt(1200.0 / (naux * nv)))


def make_system(no: int, nv: int, naux: int, seed: int, sigma: float = SIGMA, rng=None):
    """Return ``(B, eps)``: B float64 (naux, n, n) symmetric in (p,q); eps float64 (n,)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    n = no + nv
    B = rng.normal(0.0, sigma, size=(naux, n, n))
    iu, ju = np.triu_indices(n, 1)
    B[:, ju, iu] = B[:, iu, ju]
    eo = np.sort(rng.uniform(-2.0, -0.3, no))
    ev = np.sort(rng.uniform(0.1, 5.0, nv))
    return np.ascontiguousarray(B), np.concatenate([eo, ev])


def random_amplitudes(no: int, nv: int, seed: int, scale1: float = 0.02, scale2: float = 0.02):
    """Random closed-shell amplitudes: t1 (no,nv) and t2 (no,no,nv,nv) with t2[i,j,a,b] = t2[j,i,b,a]."""
    rng = np.random.default_rng(seed)
    t1 = rng.normal(0.0, scale1, size=(no, nv))
    x = rng.normal(0.0, scale2, size=(no, no, nv, nv))
    t2 = 0.5 * (x + x.transpose(1, 0, 3, 2))
    return t1, np.ascontiguousarray(t2)


def random_orthogonal(n: int, rng) -> np.ndarray:
    """Haar-random orthogonal matrix (QR of a Gaussian matrix with sign fix)."""
    q, r = np.linalg.qr(rng.normal(size=(n, n)))
    return q * np.sign(np.diag(r))


def random_symmetric_fock(eps: np.ndarray, scale: float, seed: int) -> np.ndarray:
    """diag(eps) plus a small random symmetric perturbation in every block (non-canonical, non-HF)."""
    rng = np.random.default_rng(seed)
    n = eps.shape[0]
    x = rng.normal(0.0, scale, size=(n, n))
    return np.diag(eps) + 0.5 * (x + x.T)


def single_excitation_guesses(no: int, nv: int, nstates: int, rng) -> list:
    """Distinct (i, a) pairs, one per state, drawn without replacement."""
    flat = rng.choice(no * nv, size=nstates, replace=False)
    return [(int(f // nv), int(f % nv)) for f in flat]


# The benchmark workloads (sizes and seeds) by name.
WORKLOADS = {
    "o5v20q60": dict(no=5, nv=20, naux=60, seed=0),
    "o20v180q600": dict(no=20, nv=180, naux=600, seed=1),
    "o40v360q1200": dict(no=40, nv=360, naux=1200, seed=2),
    "o30v270q900x16": dict(no=30, nv=270, naux=900, seed=3, nstates=16),
}
