"""Closed-shell, spin-adapted CCSD-form residuals and energy in T1-dressed form, FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed.  With S = 0 the transformed Hamiltonian of Eq. (eqn: sim) is H itself, and the
working equations are the ground-state CCSD projections of Eqs. (eqn:energy) and (eqn:amp)
(paper Sec. II.A) with T = T1 + T2 (Sec. II.B).  For a closed-shell singlet only the unique
amplitudes t_i^a = t_{i_alpha}^{a_alpha} and t_ij^ab = t_{i_alpha j_beta}^{a_alpha b_beta} are kept
(Supporting Information S1), and the closed-shell residuals are the matching projections
R_i^a = R_{i_alpha}^{a_alpha}, R_ij^ab = R_{i_alpha j_beta}^{a_alpha b_beta}.

How.  The textbook closed-shell equations in T1-transformed form (Helgaker, Jorgensen, Olsen,
"Molecular Electronic-Structure Theory", Sec. 13.7; Koch et al., J. Chem. Phys. 104, 4157
(1996)).  The two-electron integrals are the density-fitted ones, (pq|rs) = sum_Q B_Qpq B_Qrs,
and the dressing is the one-body transform x -> X x Y^T applied to every index pair:

    X = 1 except X_ak = -t_k^a,   Y = 1 except Y_ic = t_i^c,
    B^_Q = X B_Q Y^T,  h^ = X h Y^T,  g^_pqrs = sum_Q B^_Qpq B^_Qrs,
    F^_pq = h^_pq + sum_k (2 g^_pqkk - g^_pkkq).

The one-electron operator is h = f - sum_k (2 (pq|kk) - (pk|kq)), so that ``fock`` is exactly the
Fock matrix of the reference determinant.  Everything is formed plainly (the full dressed
virtual block g^_acbd included), with no blocking: this is a checker, not a fast code.

Pinned against ``oracle.so_ccsd`` through the spin mapping of Supporting Information S1.
"""
from __future__ import annotations

import numpy as np


def core_hamiltonian_df(B: np.ndarray, fock: np.ndarray, no: int) -> np.ndarray:
    """h = f - sum_k [2 (pq|kk) - (pk|kq)] with (pq|rs) = sum_Q B_Qpq B_Qrs."""
    dk = np.einsum("Qkk->Q", B[:, :no, :no])
    J = np.einsum("Qpq,Q->pq", B, dk)
    K = np.einsum("Qpk,Qkq->pq", B[:, :, :no], B[:, :no, :])
    return fock - (2.0 * J - K)


def dressing_matrices(t1: np.ndarray, n: int):
    """X = 1 - t1 (virtual-occupied block), Y = 1 + t1^T (occupied-virtual block) as n x n matrices."""
    no, nv = t1.shape
    X = np.eye(n)
    Y = np.eye(n)
    X[no:, :no] = -t1.T
    Y[:no, no:] = t1
    return X, Y


def dressed(B: np.ndarray, h: np.ndarray, t1: np.ndarray):
    """(B^, h^, F^) of the T1-transformed Hamiltonian."""
    no = t1.shape[0]
    n = h.shape[0]
    X, Y = dressing_matrices(t1, n)
    Bh = np.einsum("pr,Qrs,qs->Qpq", X, B, Y, optimize=True)
    hh = X @ h @ Y.T
    dk = np.einsum("Qkk->Q", Bh[:, :no, :no])
    J = np.einsum("Qpq,Q->pq", Bh, dk)
    K = np.einsum("Qpk,Qkq->pq", Bh[:, :, :no], Bh[:, :no, :])
    return Bh, hh, hh + 2.0 * J - K


def _g(Bh, P, Qs, R, S):
    """Dressed integral block g^[P,Qs,R,S] = sum_Q B^[Q,P,Qs] B^[Q,R,S]."""
    return np.einsum("Xpq,Xrs->pqrs", Bh[:, P, Qs], Bh[:, R, S], optimize=True)


def energy(B: np.ndarray, fock: np.ndarray, t1: np.ndarray, t2: np.ndarray) -> float:
    """E_corr = sum_ijab (t_ij^ab + t_i^a t_j^b)(2(ia|jb) - (ib|ja)) + 2 sum_ia f_ia t_i^a (Eq. (eqn:energy))."""
    no = t1.shape[0]
    o, v = slice(0, no), slice(no, None)
    g = np.einsum("Xia,Xjb->iajb", B[:, o, v], B[:, o, v], optimize=True)
    L = 2.0 * g - g.transpose(0, 3, 2, 1)
    tau = t2 + np.einsum("ia,jb->ijab", t1, t1)
    return float(np.einsum("ijab,iajb->", tau, L) + 2.0 * np.einsum("ia,ia->", fock[o, v], t1))


def residual(B: np.ndarray, fock: np.ndarray, t1: np.ndarray, t2: np.ndarray, terms: dict | None = None):
    """Closed-shell residuals (r1[i,a], r2[i,j,a,b]) of Eq. (eqn:amp).

    If ``terms`` is a dict it is filled with the separate contributions (each already in
    [i,a] or [i,j,a,b] layout, the doubles ones before the P_ij^ab symmetrisation where noted).
    """
    no, nv = t1.shape
    n = no + nv
    o, v = slice(0, no), slice(no, n)
    h = core_hamiltonian_df(B, fock, no)
    Bh, hh, F = dressed(B, h, t1)
    Foo, Fov, Fvo, Fvv = F[o, o], F[o, v], F[v, o], F[v, v]

    u = 2.0 * t2 - t2.transpose(0, 1, 3, 2)  # u_ij^ab = 2 t_ij^ab - t_ij^ba

    g_ovov = _g(Bh, o, v, o, v)  # equal to the undressed (kc|ld)
    g_vovo = _g(Bh, v, o, v, o)
    g_oooo = _g(Bh, o, o, o, o)
    g_oovv = _g(Bh, o, o, v, v)
    g_voov = _g(Bh, v, o, o, v)
    g_vvov = _g(Bh, v, v, o, v)
    g_ooov = _g(Bh, o, o, o, v)

    # singles: Omega_ai = sum_ckd u_ki^cd g_adkc - sum_ckl u_kl^ac g_kilc + sum_ck u_ik^ac F_kc + F_ai
    r1_a = np.einsum("kicd,adkc->ia", u, g_vvov, optimize=True)
    r1_b = -np.einsum("klac,kilc->ia", u, g_ooov, optimize=True)
    r1_c = np.einsum("ikac,kc->ia", u, Fov, optimize=True)
    r1_d = Fvo.T.copy()
    r1 = r1_a + r1_b + r1_c + r1_d

    # doubles
    r2_g = g_vovo.transpose(1, 3, 0, 2).copy()  # g_aibj -> [i,j,a,b]

    # particle-particle ladder: sum_cd t_ij^cd g_acbd, with g_acbd arranged as the matrix [(a,b),(c,d)]
    Vab_cd = np.einsum("Xac,Xbd->abcd", Bh[:, v, v], Bh[:, v, v], optimize=True).reshape(nv * nv, nv * nv)
    r2_a = (t2.reshape(no * no, nv * nv) @ Vab_cd.T).reshape(no, no, nv, nv)
    del Vab_cd

    # hole-hole ladder: sum_kl t_kl^ab (g_kilj + sum_cd t_ij^cd g_kcld)
    chi = g_oooo + np.einsum("ijcd,kcld->kilj", t2, g_ovov, optimize=True)
    r2_b = np.einsum("klab,kilj->ijab", t2, chi, optimize=True)

    # C: -1/2 sum_ck t_kj^bc (g_kiac - 1/2 sum_dl t_li^ad g_kdlc) - sum_ck t_ki^bc (g_kjac - 1/2 sum_dl t_lj^ad g_kdlc)
    Xc = g_oovv - 0.5 * np.einsum("liad,kdlc->kiac", t2, g_ovov, optimize=True)
    r2_c = -0.5 * np.einsum("kjbc,kiac->ijab", t2, Xc, optimize=True) - np.einsum("kibc,kjac->ijab", t2, Xc, optimize=True)

    # D: 1/2 sum_ck u_jk^bc (L_aikc + 1/2 sum_dl u_il^ad L_ldkc), L_pqrs = 2 g_pqrs - g_psrq
    L_aikc = 2.0 * g_voov - g_oovv.transpose(2, 1, 0, 3)  # g_acki = g_kiac
    L_ldkc = 2.0 * g_ovov - g_ovov.transpose(0, 3, 2, 1)
    Zd = L_aikc + 0.5 * np.einsum("ilad,ldkc->aikc", u, L_ldkc, optimize=True)
    r2_d = 0.5 * np.einsum("jkbc,aikc->ijab", u, Zd, optimize=True)

    # E: sum_c t_ij^ac (F_bc - sum_dkl u_kl^bd g_ldkc) - sum_k t_ik^ab (F_kj + sum_cdl u_lj^cd g_kdlc)
    Fvv_p = Fvv - np.einsum("klbd,ldkc->bc", u, g_ovov, optimize=True)
    Foo_p = Foo + np.einsum("ljcd,kdlc->kj", u, g_ovov, optimize=True)
    r2_e = np.einsum("ijac,bc->ijab", t2, Fvv_p, optimize=True) - np.einsum("ikab,kj->ijab", t2, Foo_p, optimize=True)

    cde = r2_c + r2_d + r2_e
    r2 = r2_g + r2_a + r2_b + cde + cde.transpose(1, 0, 3, 2)  # P_ij^ab X_aibj = X_aibj + X_bjai

    if terms is not None:
        terms.update(dict(r1_a=r1_a, r1_b=r1_b, r1_c=r1_c, r1_d=r1_d, r2_g=r2_g, r2_a=r2_a, r2_b=r2_b,
                          r2_c=r2_c, r2_d=r2_d, r2_e=r2_e, Fhat=F))
    return r1, r2


def mp2_energy(B: np.ndarray, eps: np.ndarray, no: int) -> float:
    """Closed-form MP2 correlation energy sum (ia|jb)[2(ia|jb) - (ib|ja)]/D_ij^ab (first-order amplitudes, Sec. II.B)."""
    o, v = slice(0, no), slice(no, None)
    g = np.einsum("Xia,Xjb->iajb", B[:, o, v], B[:, o, v], optimize=True)
    e_o, e_v = eps[o], eps[v]
    D = e_o[:, None, None, None] - e_v[None, :, None, None] + e_o[None, None, :, None] - e_v[None, None, None, :]
    return float(np.sum(g * (2.0 * g - g.transpose(0, 3, 2, 1)) / D))
