"""The ASCC transformed Hamiltonian of a 1-CSF state and its initial guess, FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed (paper Sec. II.A):

* S = (1/sqrt 2)(p_up^dagger h_up + p_dn^dagger h_dn) for a hole h (occupied) and a particle p
  (virtual) (Eq. (eqn:1CSF-S)), and the transformed Hamiltonian Hbar = e^{S^dagger} H e^{-S^dagger}
  (Eq. (eqn: sim)).  S^dagger is one-body, so Hbar stays two-body with new integral values.
* The initial cluster operator T^P(0) = beta S + gamma S^2, beta = 1, gamma = -1/2
  (Eq. (eqn:TP-guess)), as closed-shell amplitudes.
* The second ansatz (Sec. II.D): for a target reference alpha |phi_0> + S |phi_0> with a small
  Aufbau coefficient alpha, gamma = -beta^2 / 2 and (1 - beta) / beta = alpha give the "small
  beta" solve, beta = 1 / (1 + alpha); flipping the sign of the hole orbital turns alpha into
  -alpha and gives the "large beta" solve, beta = 1 / (1 - alpha).  The reported energy is the
  mean of the two.  In the unflipped orbital basis the flip is S -> -S: the transform uses
  -K and the guess's singles amplitude changes sign.

How.  With K the spatial matrix of S^dagger (K[h][p] = 1/sqrt 2, all else 0; K^2 = 0 because h != p),
e^{S^dagger} a_q^dagger e^{-S^dagger} = sum_r a_r^dagger (1 + K)_rq and e^{S^dagger} a_q e^{-S^dagger} =
sum_s (1 - K)_qs a_s, so every integral index pair (p, q) transforms as x -> (1 + K) x (1 - K):

    hbar = (1 + K) h (1 - K),   Bbar_Q = (1 + K) B_Q (1 - K),   (pq|rs)bar = sum_Q Bbar_Qpq Bbar_Qrs.

Bbar is not symmetric in (p, q); the pair-swap symmetry (pq|rs) = (rs|pq) remains.  The Fock matrix
of the reference determinant under Hbar is fbar = hbar + sum_k [2 (pq|kk)bar - (pk|kq)bar].

S^2 = 2 (1/sqrt 2)^2 p_up^dagger h_up p_dn^dagger h_dn (the same-spin squares vanish), so T^P(0)
has the singles amplitude t_h^p = beta / sqrt 2 (both spins) and the alpha-beta doubles amplitude
t_{h h}^{p p} = gamma: exactly one closed-shell entry each.

Pinned in tests/test_oracle_ascc.py against determinant-space matrix exponentials
(``oracle.bruteforce``), the spectrum of H, the 1-CSF reference of Eq. (eqn: 1csf) and the
two-electron limit, where the ASCC solution is an exact eigenstate of H.
"""
from __future__ import annotations

import numpy as np

from .cs_ccsd import core_hamiltonian_df, dressed


def s_dagger_matrix(n: int, hole: int, particle: int, sign: float = 1.0) -> np.ndarray:
    """K: the spatial matrix of S^dagger = (sign/sqrt 2) sum_spin h^dagger p, K[hole][particle] = sign/sqrt 2."""
    if not (0 <= hole < n and 0 <= particle < n and hole != particle):
        raise ValueError("hole and particle must be distinct orbitals")
    if sign not in (1.0, -1.0):
        raise ValueError("sign must be +1 or -1")
    K = np.zeros((n, n))
    K[hole, particle] = sign / np.sqrt(2.0)
    return K


def transform(B: np.ndarray, h: np.ndarray, hole: int, particle: int, sign: float = 1.0):
    """(Bbar, hbar): every index pair x -> (1 + K) x (1 - K)."""
    n = h.shape[0]
    K = s_dagger_matrix(n, hole, particle, sign)
    L, R = np.eye(n) + K, np.eye(n) - K
    Bbar = np.einsum("pr,Qrs,sq->Qpq", L, B, R, optimize=True)
    return Bbar, L @ h @ R


def transformed_inputs(B: np.ndarray, fock: np.ndarray, no: int, hole: int, particle: int, sign: float = 1.0):
    """(Bbar, fbar) for a system given by B and its reference Fock matrix ``fock`` ([n] diagonal or [n][n])."""
    n = B.shape[1]
    f = np.diag(fock) if fock.ndim == 1 else fock
    h = core_hamiltonian_df(B, f, no)
    Bbar, hbar = transform(B, h, hole, particle, sign)
    _, _, fbar = dressed(Bbar, hbar, np.zeros((no, n - no)))  # t1 = 0: fbar = hbar + 2J - K of Bbar
    return Bbar, fbar


def initial_guess(no: int, nv: int, hole: int, particle: int, beta: float = 1.0, gamma: float = -0.5):
    """Closed-shell (t1, t2) of T^P(0) = beta S + gamma S^2 (``particle`` as a full orbital index)."""
    a = particle - no
    if not (0 <= hole < no and 0 <= a < nv):
        raise ValueError("hole must be occupied and particle virtual")
    t1 = np.zeros((no, nv))
    t2 = np.zeros((no, no, nv, nv))
    t1[hole, a] = beta / np.sqrt(2.0)
    t2[hole, hole, a, a] = gamma
    return t1, t2


def two_ansatz_betas(alpha: float):
    """(beta, beta_flipped): beta of the solve with S as defined, (1 - beta)/beta = alpha, and of the
    solve with the hole sign flipped, (1 - beta)/beta = -alpha (|alpha| < 1).  For alpha > 0 the first
    is the "small beta" case and the second the "large beta" one."""
    if not abs(alpha) < 1.0:
        raise ValueError("|alpha| must be below 1")
    return 1.0 / (1.0 + alpha), 1.0 / (1.0 - alpha)


def solve_state(B, fock, no, hole, particle, beta=1.0, sign=1.0, tol_rnorm=1e-10, maxiter=400):
    """Total energy of a 1-CSF ASCC state solved from T^P(0) = beta S + gamma S^2, gamma = -beta^2/2,
    with S of the given sign (the oracle solver: Jacobi + DIIS on the closed-shell residual of Hbar)."""
    from . import cs_ccsd, solver

    f = np.diag(fock) if fock.ndim == 1 else fock
    eps = np.diag(f).copy()
    nv = B.shape[1] - no
    Bbar, fbar = transformed_inputs(B, f, no, hole, particle, sign)
    t1, t2 = initial_guess(no, nv, hole, particle, beta=sign * beta, gamma=-0.5 * beta * beta)
    res = solver.solve(lambda a, b: cs_ccsd.residual(Bbar, fbar, a, b), lambda a, b: cs_ccsd.energy(Bbar, fbar, a, b),
                       eps, t1, t2, maxiter=maxiter, tol_rnorm=tol_rnorm)
    return dict(E=reference_energy(Bbar, fbar, no) + res["E"], converged=res["converged"], t1=res["t1"],
                t2=res["t2"], iterations=res["iterations"])


def two_ansatz(B, fock, no, hole, particle, alpha, **kw):
    """The two ansatz choices for the Aufbau coefficient alpha: S as defined with beta = 1/(1 + alpha),
    and the hole sign flipped (S -> -S) with beta = 1/(1 - alpha).  The state's energy (Sec. III.A):
    the mean of the two total energies, the converged one alone if the other solve fails, none
    (converged False) if both fail."""
    b_plus, b_minus = two_ansatz_betas(alpha)
    plus = solve_state(B, fock, no, hole, particle, beta=b_plus, sign=1.0, **kw)
    minus = solve_state(B, fock, no, hole, particle, beta=b_minus, sign=-1.0, **kw)
    done = [r for r in (plus, minus) if r["converged"]]
    E = sum(r["E"] for r in done) / len(done) if done else 0.5 * (plus["E"] + minus["E"])
    return dict(plus=plus, minus=minus, E=E, converged=len(done) == 2, any_converged=bool(done),
                used=(1 if plus["converged"] else 0) | (2 if minus["converged"] else 0))


def reference_energy(B: np.ndarray, fock: np.ndarray, no: int) -> float:
    """<phi_0|H|phi_0> = sum_i (h_ii + f_ii) for a closed-shell reference (any H, Hermitian or not)."""
    f = np.diag(fock) if fock.ndim == 1 else fock
    h = core_hamiltonian_df(B, f, no)
    return float(np.trace(h[:no, :no]) + np.trace(f[:no, :no]))
