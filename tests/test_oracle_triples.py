"""The mixed-triples oracle (oracle/triples.py), pinned on the CPU:

* the explicit triples terms against brute-force determinant projections (paper Eq. (eqn:amp)) with
  generic non-symmetric integrals and generic antisymmetric T2 and T3, at a size where every
  contraction pattern is independent of the others;
* the T3 operator of the brute-force oracle against the cluster analysis of e^T|phi_0> onto triples;
* the slice against its definition (Sec. II.B.1): the triples reached by one contraction of the
  two-electron operator with the all-primary double of T^P(0) (Eq. (eqn:H1TP)), and its size;
* the closed-shell residual with the slice against projections of the transformed Hamiltonian;
* a converged ASCCSD solution: every spin-orbital single and double projection and every slice
  projection of e^{-T} Hbar e^{T} vanishes there (the whole solve checked against the definition).
"""
import itertools
from math import comb

import numpy as np
import pytest

from gen.synth_df import converging_sigma, make_system, random_amplitudes
from oracle import ascc, cs_ccsd, triples
from oracle.bruteforce import BruteForce, closed_shell_to_so, so_maps, so_to_closed_shell
from oracle.so_ccsd import so_fock_and_antisym


def _eri(B):
    return np.einsum("Qpq,Qrs->pqrs", B, B)


def _generic(o, v, seed):
    """Non-symmetric integrals, the one-body operator and the reference Fock matrix they imply."""
    rng = np.random.default_rng(seed)
    n = o + v
    B = 0.3 * rng.standard_normal((6, n, n))
    h = 0.3 * rng.standard_normal((n, n)) + np.diag(np.arange(n) - 2.0)
    eri = _eri(B)
    fock = h + 2.0 * np.einsum("pqkk->pq", eri[:, :, :o, :o]) - np.einsum("pkkq->pq", eri[:, :o, :o, :])
    return h, eri, fock, rng


@pytest.mark.parametrize("o,v,seed", [(3, 3, 71), (2, 3, 72)])
def test_triples_terms_equal_brute_force_projections(o, v, seed):
    """R3, and the T3 parts of R1 and R2, from the explicit terms equal the projections.  At o = v = 3
    the 19 antisymmetrised patterns of R3 are linearly independent, so no error in one factor can
    be compensated by another."""
    h, eri, fock, rng = _generic(o, v, seed)
    bf = BruteForce(h, eri, o, v)
    f, g = so_fock_and_antisym(fock, eri, o, v)
    no_, nv_ = 2 * o, 2 * v
    t1 = np.zeros((no_, nv_))
    t2 = triples.antisym2(rng.standard_normal((no_, no_, nv_, nv_))) / 4.0
    t3 = triples.antisym3(rng.standard_normal((no_,) * 3 + (nv_,) * 3)) / 36.0
    _, r1, r2, r3 = bf.projections(t1, t2, t3, triples=True)
    _, q1, q2 = bf.projections(t1, t2)
    a1, a2, a3 = triples.t3_terms(f, g, t2, t3, no_)
    assert np.abs(a3 - r3).max() < 1e-11 * max(1.0, np.abs(r3).max())
    assert np.abs(a1 - (r1 - q1)).max() < 1e-12
    assert np.abs(a2 - (r2 - q2)).max() < 1e-12


def test_a_wrong_triples_factor_is_caught():
    """Halving the T2 T3 ring term (a plausible slip) breaks the equality."""
    o, v = 3, 3
    h, eri, fock, rng = _generic(o, v, 73)
    bf = BruteForce(h, eri, o, v)
    f, g = so_fock_and_antisym(fock, eri, o, v)
    no_, nv_ = 2 * o, 2 * v
    t2 = triples.antisym2(rng.standard_normal((no_, no_, nv_, nv_))) / 4.0
    t3 = triples.antisym3(rng.standard_normal((no_,) * 3 + (nv_,) * 3)) / 36.0
    _, _, _, r3 = bf.projections(np.zeros((no_, nv_)), t2, t3, triples=True)
    _, _, a3 = triples.t3_terms(f, g, t2, t3, no_)
    ring = triples.antisym3(0.25 * np.einsum("mnef,miea,njkfbc->ijkabc", g[:no_, :no_, no_:, no_:], t2, t3))
    assert np.abs(a3 - r3).max() < 1e-10
    assert np.abs(a3 - 0.5 * ring - r3).max() > 1e-3


@pytest.mark.parametrize("o,v,seed", [(2, 3, 74), (3, 2, 75)])
def test_t3_operator_gives_the_cluster_analysis(o, v, seed):
    """The triples part of e^T|phi_0> is C3 = T3 + T1 T2 + T1^3/6: for the antisymmetric tensors,
    c_ijk^abc = t_ijk^abc + A3[t_i^a t_jk^bc]/4 + A3[t_i^a t_j^b t_k^c]/6."""
    h, eri, fock, rng = _generic(o, v, seed)
    bf = BruteForce(h, eri, o, v)
    no_, nv_ = 2 * o, 2 * v
    t1 = rng.standard_normal((no_, nv_))
    t2 = triples.antisym2(rng.standard_normal((no_, no_, nv_, nv_))) / 4.0
    t3 = triples.antisym3(rng.standard_normal((no_,) * 3 + (nv_,) * 3)) / 36.0
    psi = bf.exp_T(t1, t2, bf.ref, 1.0, t3)
    c3 = np.zeros_like(t3)
    for occ in itertools.combinations(range(no_), 3):
        for vir in itertools.combinations(range(nv_), 3):
            c3[occ + vir] = bf.triple(*occ, *vir) @ psi
    want = t3 + triples.antisym3(np.einsum("ia,jkbc->ijkabc", t1, t2)) / 4.0 \
        + triples.antisym3(np.einsum("ia,jb,kc->ijkabc", t1, t1, t1)) / 6.0
    for occ in itertools.combinations(range(no_), 3):
        for vir in itertools.combinations(range(nv_), 3):
            assert abs(c3[occ + vir] - want[occ + vir]) < 1e-12


def _slice_size(o, v):
    """Both hole spin orbitals emptied and at least one particle spin orbital filled, or one hole
    spin orbital emptied and both particle spin orbitals filled, at the reference's S_z."""
    a = 2 * (o - 1) * (v * comb(v, 2) - (v - 1) * comb(v - 1, 2))
    b = 2 * (v - 1) * ((o - 1) ** 2 + comb(o - 1, 2))
    return a + b


@pytest.mark.parametrize("o,v", [(1, 3), (2, 2), (2, 5), (3, 3), (4, 2), (5, 7), (20, 180)])
def test_slice_size(o, v):
    if o * v <= 35:
        assert len(triples.slice_triples(o, v, 0, o)) == _slice_size(o, v)
    n = _slice_size(o, v)
    assert n <= 4 * (o * v * v + o * o * v)  # O(o^2 v + o v^2)
    if o == 1:
        assert n == 0


@pytest.mark.parametrize("o,v,hole,particle,seed", [(3, 3, 1, 4, 76), (2, 4, 0, 3, 77)])
def test_slice_is_what_one_contraction_reaches(o, v, hole, particle, seed):
    """<mu3| [W, T_pp] |phi_0> for the two-electron operator W of generic (non-symmetric) integrals and
    the all-primary double T_pp of T^P(0) is non-zero exactly on the slice (Eq. (eqn:H1TP))."""
    rng = np.random.default_rng(seed)
    n = o + v
    B = 0.5 * rng.standard_normal((5, n, n))
    bf = BruteForce(np.zeros((n, n)), _eri(B), o, v)
    t2 = np.zeros((o, o, v, v))
    t2[hole, hole, particle - o, particle - o] = -0.5
    z1, t2so = closed_shell_to_so(np.zeros((o, v)), t2)
    comm = bf.apply_H(bf.apply_T(z1, t2so, bf.ref)) - bf.apply_T(z1, t2so, bf.apply_H(bf.ref))
    reached = set()
    for occ in itertools.combinations(range(2 * o), 3):
        for vir in itertools.combinations(range(2 * v), 3):
            if abs(bf.triple(*occ, *vir) @ comm) > 1e-12:
                reached.add(occ + vir)
    assert reached == set(triples.slice_triples(o, v, hole, particle))


@pytest.mark.parametrize("o,v,Q,seed,hole,particle", [(2, 3, 7, 78, 1, 3), (3, 3, 8, 79, 0, 4)])
def test_closed_shell_residual_with_slice_equals_projections(o, v, Q, seed, hole, particle):
    """Closed-shell singles and doubles with the T3 couplings, and the slice residual, of the
    non-symmetric Hbar (T1 dressing included) equal the brute-force projections."""
    B, eps = make_system(o, v, Q, seed, sigma=0.3)
    Bbar, fbar = ascc.transformed_inputs(B, eps, o, hole, particle)
    t1, t2 = random_amplitudes(o, v, seed, scale1=0.1, scale2=0.1)
    tri = triples.slice_triples(o, v, hole, particle)
    rng = np.random.default_rng(seed)
    t3 = triples.unpack(0.1 * rng.standard_normal(len(tri)), tri, o, v)
    mask = triples.slice_mask(o, v, hole, particle)
    r1, r2, r3 = triples.residual(Bbar, fbar, t1, t2, t3, mask)
    h = cs_ccsd.core_hamiltonian_df(Bbar, fbar, o)
    t1so, t2so = closed_shell_to_so(t1, t2)
    E, q1, q2, q3 = BruteForce(h, _eri(Bbar), o, v).projections(t1so, t2so, t3, triples=True)
    R1, R2 = so_to_closed_shell(q1, q2, o, v)
    assert np.abs(r1 - R1).max() < 1e-11
    assert np.abs(r2 - R2).max() < 1e-11
    assert np.abs(r3 - np.where(mask, q3, 0.0)).max() < 1e-11
    assert np.abs(np.where(mask, q3, 0.0)).max() > 1e-3


def _spin_flip(no, nv):
    """Spin-orbital permutation (occupied, virtual) that exchanges alpha and beta."""
    spatial, spin = so_maps(no, nv)
    occ = [no + i if i < no else i - no for i in range(2 * no)]
    vir = [nv + a if a < nv else a - nv for a in range(2 * nv)]
    return np.array(occ), np.array(vir)


@pytest.mark.parametrize("o,v,Q,seed,hole,particle,width", [(3, 3, 8, 81, 2, 3, 0.5), (2, 4, 8, 84, 1, 3, 1.0)])
def test_asccsd_solution_satisfies_every_projection(o, v, Q, seed, hole, particle, width):
    """At the converged ASCCSD solution every spin-orbital single and double projection and every slice
    projection of e^{-T} Hbar e^{T}|phi_0> vanishes, the energy is the reference one, the triples are
    symmetric under the exchange of alpha and beta, and they shift the energy."""
    B, eps = make_system(o, v, Q, seed, sigma=width * converging_sigma(v, Q))
    res = triples.solve_state(B, eps, o, hole, particle, tol_rnorm=1e-11)
    assert res["converged"]
    t1so, t2so = closed_shell_to_so(res["t1"], res["t2"])
    h = cs_ccsd.core_hamiltonian_df(res["Bbar"], res["fbar"], o)
    E, q1, q2, q3 = BruteForce(h, _eri(res["Bbar"]), o, v).projections(t1so, t2so, res["t3"], triples=True)
    mask = triples.slice_mask(o, v, hole, particle)
    assert np.abs(q1).max() < 1e-9
    assert np.abs(q2).max() < 1e-9
    assert np.abs(np.where(mask, q3, 0.0)).max() < 1e-9
    assert abs(E - res["E"]) < 1e-10
    po, pv = _spin_flip(o, v)
    t3 = res["t3"]
    assert np.abs(t3 - t3[np.ix_(po, po, po, pv, pv, pv)]).max() < 1e-9
    assert np.abs(t3).max() > 1e-4
    plain = ascc.solve_state(B, eps, o, hole, particle, tol_rnorm=1e-11)
    assert plain["converged"] and abs(plain["E"] - res["E"]) > 1e-6


def test_two_electrons_have_no_mixed_triples():
    """With o = 1 the slice is empty and ASCCSD is ASCC."""
    o, v, Q, hole, particle = 1, 4, 7, 0, 2
    B, eps = make_system(o, v, Q, 82, sigma=converging_sigma(v, Q))
    a = triples.solve_state(B, eps, o, hole, particle, tol_rnorm=1e-11)
    b = ascc.solve_state(B, eps, o, hole, particle, tol_rnorm=1e-11)
    assert a["triples"] == [] and a["converged"] and b["converged"]
    assert abs(a["E"] - b["E"]) < 1e-10
