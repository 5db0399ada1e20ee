"""Determinant-space evaluation of the coupled-cluster energy and residuals by definition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What it computes (paper Sec. II.A):

* the exponential ansatz with T = T1 + T2 (+ T3), where T_N carries the prefactor (1/N!)^2 and
  the operator string a^dagger b^dagger ... j i (Eq. (eqn: CC equation) and the T_N definition);
* the energy <phi_0| e^{-T} H e^{T} |phi_0> (Eq. (eqn:energy));
* the residuals <mu| e^{-T} H e^{T} |phi_0> for every singly, doubly and (optionally) triply
  excited determinant mu (Eq. (eqn:amp)); with S = 0 the transformed Hamiltonian is H itself
  (Eq. (eqn: sim)).  Triples enter the 1-CSF excited-state ansatz through the mixed slice
  T^M_3' (Sec. II.B.1); here T3 is a full antisymmetric tensor, zero wherever the caller wants.

Everything is done with explicit second-quantised operators on bit-string determinants, so
nothing here depends on a factorisation of the CC equations.  Cost grows as the number of
determinants C(2n, 2o): use it for no <= 3, nv <= 4 or so.

Spin-orbital numbering (used across ``oracle``): occupied alpha i -> i, occupied beta i ->
no + i, virtual alpha a -> 2 no + a, virtual beta a -> 2 no + nv + a.  The reference
determinant fills spin orbitals 0 .. 2 no - 1.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def so_maps(no: int, nv: int):
    """Spatial index and spin (0 alpha, 1 beta) of every spin orbital, in the numbering above."""
    n = no + nv
    spatial = np.empty(2 * n, dtype=np.int64)
    spin = np.empty(2 * n, dtype=np.int64)
    for i in range(no):
        spatial[i], spin[i] = i, 0
        spatial[no + i], spin[no + i] = i, 1
    for a in range(nv):
        spatial[2 * no + a], spin[2 * no + a] = no + a, 0
        spatial[2 * no + nv + a], spin[2 * no + nv + a] = no + a, 1
    return spatial, spin


def core_hamiltonian(eri: np.ndarray, fock: np.ndarray, no: int) -> np.ndarray:
    """One-electron operator h whose reference Fock matrix is ``fock``: h = f - sum_k [2 (pq|kk) - (pk|kq)]."""
    occ = slice(0, no)
    J = np.einsum("pqkk->pq", eri[:, :, occ, occ])
    K = np.einsum("pkkq->pq", eri[:, occ, occ, :])
    return fock - (2.0 * J - K)


def spin_orbital_integrals(h: np.ndarray, eri: np.ndarray, no: int, nv: int):
    """Spin-orbital h_PQ and physicist's <PQ|RS> = (PR|QS) delta(s_P,s_R) delta(s_Q,s_S)."""
    spatial, spin = so_maps(no, nv)
    hso = h[np.ix_(spatial, spatial)] * (spin[:, None] == spin[None, :])
    chem = eri[np.ix_(spatial, spatial, spatial, spatial)]  # (PQ|RS) in spatial values
    same = spin[:, None] == spin[None, :]
    chem = chem * same[:, :, None, None] * same[None, None, :, :]
    phys = chem.transpose(0, 2, 1, 3)  # <PQ|RS> = (PR|QS)
    return hso, np.ascontiguousarray(phys)


class DeterminantSpace:
    """All determinants of ``nelec`` electrons in ``nso`` spin orbitals, and a^dagger_p a_q on them."""

    def __init__(self, nso: int, nelec: int):
        self.nso = nso
        self.nelec = nelec
        self.dets = [sum(1 << p for p in occ) for occ in itertools.combinations(range(nso), nelec)]
        self.index = {d: k for k, d in enumerate(self.dets)}
        self.dim = len(self.dets)
        self._E = {}

    @staticmethod
    def _sign_below(det: int, p: int) -> int:
        return -1 if bin(det & ((1 << p) - 1)).count("1") % 2 else 1

    def apply_excitation(self, det: int, p: int, q: int):
        """a^dagger_p a_q |det> as (sign, new_det) or None."""
        if not (det >> q) & 1:
            return None
        s = self._sign_below(det, q)
        d1 = det & ~(1 << q)
        if (d1 >> p) & 1:
            return None
        s *= self._sign_below(d1, p)
        return s, d1 | (1 << p)

    def E(self, p: int, q: int) -> sp.csr_matrix:
        """Sparse matrix of a^dagger_p a_q."""
        key = (p, q)
        if key not in self._E:
            rows, cols, vals = [], [], []
            for k, d in enumerate(self.dets):
                r = self.apply_excitation(d, p, q)
                if r is not None:
                    rows.append(self.index[r[1]])
                    cols.append(k)
                    vals.append(float(r[0]))
            self._E[key] = sp.csr_matrix((vals, (rows, cols)), shape=(self.dim, self.dim))
        return self._E[key]

    def basis_vector(self, occupied) -> np.ndarray:
        v = np.zeros(self.dim)
        v[self.index[sum(1 << p for p in occupied)]] = 1.0
        return v


class BruteForce:
    """H, T and e^{-T} H e^{T} |phi_0> in the full determinant space of a small system."""

    def __init__(self, h: np.ndarray, eri: np.ndarray, no: int, nv: int):
        self.no, self.nv = no, nv
        self.nso = 2 * (no + nv)
        self.hso, self.g = spin_orbital_integrals(h, eri, no, nv)
        self.space = DeterminantSpace(self.nso, 2 * no)
        self.ref = self.space.basis_vector(range(2 * no))
        nso = self.nso
        # a^dagger_p a^dagger_q a_s a_r = E_pr E_qs - delta_qr E_ps, so
        # H = sum_ps (h_ps - 1/2 sum_q <pq|qs>) E_ps + 1/2 sum_pqrs <pq|rs> E_pr E_qs.
        self.hmod = self.hso - 0.5 * np.einsum("pqqs->ps", self.g)
        self._Es = [[self.space.E(p, q) for q in range(nso)] for p in range(nso)]

    def apply_H(self, psi: np.ndarray) -> np.ndarray:
        nso = self.nso
        phi = np.stack([np.stack([self._Es[q][s] @ psi for s in range(nso)]) for q in range(nso)])  # [q,s,D]
        w = 0.5 * np.einsum("pqrs,qsD->prD", self.g, phi) + self.hmod[:, :, None] * psi[None, None, :]
        out = np.zeros_like(psi)
        for p in range(nso):
            for r in range(nso):
                out += self._Es[p][r] @ w[p, r]
        return out

    def apply_T(self, t1so: np.ndarray, t2so: np.ndarray, psi: np.ndarray) -> np.ndarray:
        """T psi with T = sum_ia t_i^a a^dagger_a a_i + 1/4 sum_ijab t_ij^ab a^dagger_a a^dagger_b a_j a_i.

        a^dagger_a a^dagger_b a_j a_i = E_ai E_bj (i, j occupied; a, b virtual).
        """
        nocc = 2 * self.no
        nvir = self.nso - nocc
        phi = np.stack([np.stack([self._Es[nocc + b][j] @ psi for j in range(nocc)]) for b in range(nvir)])  # [b,j,D]
        w = 0.25 * np.einsum("ijab,bjD->aiD", t2so, phi) + t1so.T[:, :, None] * psi[None, None, :]
        out = np.zeros_like(psi)
        for a in range(nvir):
            for i in range(nocc):
                out += self._Es[nocc + a][i] @ w[a, i]
        return out

    def apply_T3(self, t3so: np.ndarray, psi: np.ndarray) -> np.ndarray:
        """T3 psi with T3 = 1/36 sum_ijkabc t_ijk^abc a^dagger_a a^dagger_b a^dagger_c a_k a_j a_i.

        a^dagger_a a^dagger_b a^dagger_c a_k a_j a_i = E_ai E_bj E_ck (all occupied i, j, k and
        virtual a, b, c), so T3 = 1/36 sum t_ijk^abc E_ai (E_bj (E_ck psi)).
        """
        nocc = 2 * self.no
        nvir = self.nso - nocc
        E = self._Es
        p1 = [[E[nocc + c][k] @ psi for k in range(nocc)] for c in range(nvir)]  # [c][k]
        p2 = np.stack([np.stack([np.stack([np.stack([E[nocc + b][j] @ p1[c][k] for k in range(nocc)])
                                           for c in range(nvir)]) for j in range(nocc)]) for b in range(nvir)])
        w = np.einsum("ijkabc,bjckD->aiD", t3so, p2) / 36.0
        out = np.zeros_like(psi)
        for a in range(nvir):
            for i in range(nocc):
                out += E[nocc + a][i] @ w[a, i]
        return out

    def exp_T(self, t1so, t2so, psi, sign: float = 1.0, t3so=None) -> np.ndarray:
        """exp(sign*T) psi by its finite Taylor series (T is nilpotent)."""
        total = psi.copy()
        term = psi.copy()
        for k in range(1, 2 * self.no + 2):
            nxt = self.apply_T(t1so, t2so, term)
            if t3so is not None:
                nxt = nxt + self.apply_T3(t3so, term)
            term = sign * nxt / k
            if not np.any(term):
                break
            total += term
        return total

    def similarity_vector(self, t1so, t2so, t3so=None) -> np.ndarray:
        """e^{-T} H e^{T} |phi_0>."""
        v = self.exp_T(t1so, t2so, self.ref, 1.0, t3so)
        v = self.apply_H(v)
        return self.exp_T(t1so, t2so, v, -1.0, t3so)

    def triple(self, i, j, k, a, b, c) -> np.ndarray:
        """|phi_ijk^abc> = a^dagger_a a^dagger_b a^dagger_c a_k a_j a_i |phi_0> (spin-orbital indices,
        occupied i, j, k from 0 and virtual a, b, c from 0)."""
        nocc = 2 * self.no
        E = self._Es
        return E[nocc + a][i] @ (E[nocc + b][j] @ (E[nocc + c][k] @ self.ref))

    def triples_projections(self, t1so, t2so, t3so=None, v=None) -> np.ndarray:
        """R_ijk^abc = <phi_ijk^abc| e^{-T} H e^{T} |phi_0> for every triple, as a full antisymmetric tensor."""
        if v is None:
            v = self.similarity_vector(t1so, t2so, t3so)
        nocc = 2 * self.no
        nvir = self.nso - nocc
        r3 = np.zeros((nocc,) * 3 + (nvir,) * 3)
        for occ in itertools.combinations(range(nocc), 3):
            for vir in itertools.combinations(range(nvir), 3):
                x = float(self.triple(*occ, *vir) @ v)
                for po, so in _signed_permutations(occ):
                    for pv, sv in _signed_permutations(vir):
                        r3[po + pv] = so * sv * x
        return r3

    def projections(self, t1so, t2so, t3so=None, triples: bool = False):
        """Energy and spin-orbital residuals R_i^a, R_ij^ab (antisymmetric) by projection, and
        R_ijk^abc as well when ``triples`` is set.

        |phi_i^a> = a^dagger_a a_i |phi_0>, |phi_ij^ab> = a^dagger_a a^dagger_b a_j a_i |phi_0>.
        """
        v = self.similarity_vector(t1so, t2so, t3so)
        nocc = 2 * self.no
        nvir = self.nso - nocc
        E = float(self.ref @ v)
        r1 = np.zeros((nocc, nvir))
        r2 = np.zeros((nocc, nocc, nvir, nvir))
        for i in range(nocc):
            for a in range(nvir):
                r1[i, a] = (self._Es[nocc + a][i] @ self.ref) @ v
        for i in range(nocc):
            for j in range(i + 1, nocc):
                for a in range(nvir):
                    for b in range(a + 1, nvir):
                        mu = self._Es[nocc + a][i] @ (self._Es[nocc + b][j] @ self.ref)
                        x = float(mu @ v)
                        r2[i, j, a, b] = x
                        r2[j, i, a, b] = -x
                        r2[i, j, b, a] = -x
                        r2[j, i, b, a] = x
        if triples:
            return E, r1, r2, self.triples_projections(t1so, t2so, t3so, v)
        return E, r1, r2

    def hamiltonian_matrix(self) -> np.ndarray:
        """Dense H (only for very small spaces)."""
        D = self.space.dim
        H = np.empty((D, D))
        for k in range(D):
            e = np.zeros(D)
            e[k] = 1.0
            H[:, k] = self.apply_H(e)
        return H

    def s_squared_matrix(self) -> np.ndarray:
        """Dense S^2 = S_- S_+ + S_z (S_z + 1) in the same space."""
        no, nv = self.no, self.nv
        spatial, spin = so_maps(no, nv)
        n = no + nv
        alpha = {int(spatial[p]): p for p in range(self.nso) if spin[p] == 0}
        beta = {int(spatial[p]): p for p in range(self.nso) if spin[p] == 1}
        Splus = sum(self._Es[alpha[s]][beta[s]] for s in range(n))
        Sminus = sum(self._Es[beta[s]][alpha[s]] for s in range(n))
        Sz = 0.5 * sum(self._Es[alpha[s]][alpha[s]] - self._Es[beta[s]][beta[s]] for s in range(n))
        S2 = Sminus @ Splus + Sz @ Sz + Sz
        return S2.toarray()


def _signed_permutations(idx):
    """Every ordering of ``idx`` with the sign of the permutation that produces it."""
    out = []
    for perm in itertools.permutations(range(len(idx))):
        inv = sum(1 for x in range(len(perm)) for y in range(x + 1, len(perm)) if perm[x] > perm[y])
        out.append((tuple(idx[q] for q in perm), -1 if inv % 2 else 1))
    return out


def closed_shell_to_so(t1: np.ndarray, t2: np.ndarray):
    """Spin-orbital amplitudes from closed-shell singlet ones (Supporting Information S1).

    t_{i_s}^{a_s} = t_i^a for both spins; t_{i_alpha j_beta}^{a_alpha b_beta} = t_ij^ab;
    t_{i_alpha j_alpha}^{a_alpha b_alpha} = t_ij^ab - t_ji^ab (and the same for beta); all other
    entries follow from antisymmetry in (i,j) and in (a,b), or vanish by spin.
    """
    no, nv = t1.shape
    nocc, nvir = 2 * no, 2 * nv
    t1so = np.zeros((nocc, nvir))
    t2so = np.zeros((nocc, nocc, nvir, nvir))
    A, B = slice(0, no), slice(no, nocc)  # occupied alpha / beta
    a_, b_ = slice(0, nv), slice(nv, nvir)  # virtual alpha / beta
    t1so[A, a_] = t1
    t1so[B, b_] = t1
    same = t2 - t2.transpose(1, 0, 2, 3)
    t2so[A, A, a_, a_] = same
    t2so[B, B, b_, b_] = same
    t2so[A, B, a_, b_] = t2
    t2so[B, A, b_, a_] = t2  # complete spin flip of the alpha-beta block
    t2so[A, B, b_, a_] = -t2.transpose(0, 1, 3, 2)
    t2so[B, A, a_, b_] = -t2.transpose(1, 0, 2, 3)
    return t1so, t2so


def so_to_closed_shell(r1so: np.ndarray, r2so: np.ndarray, no: int, nv: int):
    """Closed-shell residuals as the alpha / alpha-beta projections: R_i^a = R_{i_a}^{a_a}, R_ij^ab = R_{i_a j_b}^{a_a b_b}."""
    return r1so[:no, :nv].copy(), r2so[:no, no:, :nv, nv:].copy()
