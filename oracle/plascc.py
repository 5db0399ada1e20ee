"""PLASCC, the partially linearised ASCC residual, FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed (paper Sec. II.C, with the amplitude classes of Sec. II.B, Eq. (eqn: pnm split)):

* the primary orbitals are those whose indices appear in S: the hole h and the particle p of a
  1-CSF state;
* T^P holds the amplitudes whose indices are all primary, T^N those with no primary index, and
  T^M the mixed ones, with both primary and non-primary indices;
* PLASCC removes from the amplitude equations every term that carries two or more powers of T^M,
  where T^M_1 is not counted (the singles stay in to all orders); the same removal, with the same
  primaries, applies to the ground-state equations.

How.  With T1 held fixed, the doubles residual of the closed-shell equations is a polynomial of
degree two in T2 (H is two-body, so a doubles projection connects at most two T2), and the
singles residual and the energy are of degree one.  Writing T2 = T2^R + lam T2^M (R = P + N), the
terms with two powers of T2^M make up the lam^2 coefficient c of

    R2(lam) = a + b lam + c lam^2,    c = [R2(1) + R2(-1)] / 2 - R2(0),

and PLASCC's doubles residual is R2(1) - c = a + b.  R1 and the energy are unchanged.

A closed-shell amplitude t2[i][j][a][b] (the alpha-beta one, Supporting Information S1) is mixed
when its spatial indices contain h (among i, j) or p (among a, b) and are not all primary; the
same-spin amplitudes t2[ijab] - t2[ijba] share the index set, so one mask serves every spin block.

Pinned in tests/test_oracle_plascc.py: against brute-force determinant projections with the mixed
set taken in the spin-orbital basis, the degree-two structure, the reductions to CCSD (no mixed
amplitudes) and to a linear doubles equation (only mixed amplitudes, T1 = 0), and size
consistency of converged ground-state energies over non-interacting fragments.
"""
from __future__ import annotations

import numpy as np

from . import cs_ccsd


def mixed_mask(no: int, nv: int, hole: int, particle: int) -> np.ndarray:
    """Boolean [o][o][v][v]: True where t2[i][j][a][b] belongs to T^M (``particle`` a full orbital index)."""
    a0 = particle - no
    if not (0 <= hole < no and 0 <= a0 < nv):
        raise ValueError("hole must be occupied and particle virtual")
    i = np.arange(no)[:, None, None, None]
    j = np.arange(no)[None, :, None, None]
    a = np.arange(nv)[None, None, :, None]
    b = np.arange(nv)[None, None, None, :]
    any_primary = (i == hole) | (j == hole) | (a == a0) | (b == a0)
    all_primary = (i == hole) & (j == hole) & (a == a0) & (b == a0)
    return np.asarray(any_primary & ~all_primary)


def split(t2: np.ndarray, hole: int, particle: int):
    """(T2^R, T2^M): the non-mixed and the mixed parts of the doubles."""
    no, _, nv, _ = t2.shape
    m = mixed_mask(no, nv, hole, particle)
    tM = np.where(m, t2, 0.0)
    return t2 - tM, tM


def mixed_quadratic(B: np.ndarray, fock: np.ndarray, t1: np.ndarray, t2: np.ndarray, hole: int, particle: int):
    """c: the part of the doubles residual with two powers of T2^M."""
    tR, tM = split(t2, hole, particle)
    _, r_plus = cs_ccsd.residual(B, fock, t1, tR + tM)
    _, r_minus = cs_ccsd.residual(B, fock, t1, tR - tM)
    _, r_zero = cs_ccsd.residual(B, fock, t1, tR)
    return 0.5 * (r_plus + r_minus) - r_zero


def residual(B: np.ndarray, fock: np.ndarray, t1: np.ndarray, t2: np.ndarray, hole: int, particle: int):
    """(R1, R2) of PLASCC: the closed-shell residual without its terms quadratic in T2^M."""
    r1, r2 = cs_ccsd.residual(B, fock, t1, t2)
    return r1, r2 - mixed_quadratic(B, fock, t1, t2, hole, particle)


def energy(B: np.ndarray, fock: np.ndarray, t1: np.ndarray, t2: np.ndarray) -> float:
    """The energy is linear in T2, so no term of it carries two powers of T^M: that of CCSD."""
    return cs_ccsd.energy(B, fock, t1, t2)
