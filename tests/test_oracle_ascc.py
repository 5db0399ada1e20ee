"""The ASCC transformed Hamiltonian of the oracle (oracle/ascc.py), pinned on the CPU:

* against the definition Hbar = e^{S^dagger} H e^{-S^dagger} (paper Eq. (eqn: sim)) evaluated with
  dense matrix exponentials in the full determinant space;
* against the spectrum of H, which a similarity transform preserves (Sec. II.A);
* the initial guess T^P(0) = S - S^2/2 (Eq. (eqn:TP-guess)) against the 1-CSF reference S|phi_0>
  of Eq. (eqn: 1csf);
* the closed-shell residual of the non-symmetric Hbar against brute-force projections;
* the two-electron limit: a converged ASCC solution is an exact eigenstate of H.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from gen.synth_df import converging_sigma, make_system, random_amplitudes
from oracle import ascc, cs_ccsd, solver
from oracle.bruteforce import BruteForce, closed_shell_to_so, so_maps, so_to_closed_shell


def _eri(B):
    return np.einsum("Qpq,Qrs->pqrs", B, B)


def _spin_orbital(no, nv, spatial_index, spin):
    sp, sn = so_maps(no, nv)
    return int(np.flatnonzero((sp == spatial_index) & (sn == spin))[0])


def _s_ops(bf, no, nv, hole, particle):
    """Dense S and S^dagger of Eq. (eqn:1CSF-S) in the determinant space of ``bf``."""
    s = 1.0 / np.sqrt(2.0)
    S = sum(s * bf.space.E(_spin_orbital(no, nv, particle, sg), _spin_orbital(no, nv, hole, sg)) for sg in (0, 1))
    Sd = sum(s * bf.space.E(_spin_orbital(no, nv, hole, sg), _spin_orbital(no, nv, particle, sg)) for sg in (0, 1))
    return S.toarray(), Sd.toarray()


CASES = [(1, 3, 5, 31, 0, 1), (2, 3, 8, 32, 1, 2), (2, 3, 7, 33, 0, 4), (3, 2, 6, 34, 2, 3)]


@pytest.mark.parametrize("o,v,Q,seed,hole,particle", CASES)
def test_transformed_integrals_are_the_similarity_transform(o, v, Q, seed, hole, particle):
    B, eps = make_system(o, v, Q, seed, sigma=0.3)
    h = cs_ccsd.core_hamiltonian_df(B, np.diag(eps), o)
    bf = BruteForce(h, _eri(B), o, v)
    H = bf.hamiltonian_matrix()
    _, Sd = _s_ops(bf, o, v, hole, particle)
    Hbar_def = sla.expm(Sd) @ H @ sla.expm(-Sd)
    Bbar, hbar = ascc.transform(B, h, hole, particle)
    assert np.abs(Bbar - Bbar.transpose(0, 2, 1)).max() > 1e-3  # really not symmetric
    Hbar = BruteForce(hbar, _eri(Bbar), o, v).hamiltonian_matrix()
    assert np.abs(Hbar - Hbar_def).max() < 1e-12
    # the spectrum is that of H
    ev_h = np.sort(np.linalg.eigvalsh(H))
    ev_bar = np.sort(np.linalg.eigvals(Hbar).real)
    assert np.abs(ev_h - ev_bar).max() < 1e-9


def test_a_wrong_transform_is_caught():
    """Transforming with (1 + K) on both sides (a plausible slip) breaks the definition."""
    o, v, Q, seed, hole, particle = 2, 3, 8, 32, 1, 2
    B, eps = make_system(o, v, Q, seed, sigma=0.3)
    h = cs_ccsd.core_hamiltonian_df(B, np.diag(eps), o)
    bf = BruteForce(h, _eri(B), o, v)
    _, Sd = _s_ops(bf, o, v, hole, particle)
    Hbar_def = sla.expm(Sd) @ bf.hamiltonian_matrix() @ sla.expm(-Sd)
    n = o + v
    L = np.eye(n) + ascc.s_dagger_matrix(n, hole, particle)
    Bw = np.einsum("pr,Qrs,sq->Qpq", L, B, L)
    Hw = BruteForce(L @ h @ L, _eri(Bw), o, v).hamiltonian_matrix()
    assert np.abs(Hw - Hbar_def).max() > 1e-3


@pytest.mark.parametrize("o,v,hole,particle", [(1, 3, 0, 1), (2, 3, 1, 2), (2, 2, 0, 3)])
def test_initial_guess_gives_the_1csf_reference(o, v, hole, particle):
    """e^{-S^dagger} e^{T^P(0)} |phi_0> = S |phi_0> for T^P(0) = S - S^2/2 (Eqs. (eqn: ogascc), (eqn: 1csf))."""
    B, eps = make_system(o, v, 4, 40, sigma=0.3)
    h = cs_ccsd.core_hamiltonian_df(B, np.diag(eps), o)
    bf = BruteForce(h, _eri(B), o, v)
    S, Sd = _s_ops(bf, o, v, hole, particle)
    t1, t2 = ascc.initial_guess(o, v, hole, particle)
    t1so, t2so = closed_shell_to_so(t1, t2)
    psi = sla.expm(-Sd) @ bf.exp_T(t1so, t2so, bf.ref)
    target = S @ bf.ref
    assert np.abs(psi - target).max() < 1e-12
    assert np.linalg.norm(target) > 0.99  # S|phi_0> is a normalised singlet CSF


@pytest.mark.parametrize("o,v,Q,seed,hole,particle", CASES)
def test_closed_shell_residual_of_the_transformed_hamiltonian(o, v, Q, seed, hole, particle):
    """The dressed closed-shell oracle, fed the non-symmetric Bbar and fbar, equals the projections."""
    B, eps = make_system(o, v, Q, seed, sigma=0.3)
    Bbar, fbar = ascc.transformed_inputs(B, eps, o, hole, particle)
    h = cs_ccsd.core_hamiltonian_df(B, np.diag(eps), o)
    _, hbar = ascc.transform(B, h, hole, particle)
    assert np.abs(cs_ccsd.core_hamiltonian_df(Bbar, fbar, o) - hbar).max() < 1e-12
    t1, t2 = random_amplitudes(o, v, seed + 60, 0.1, 0.1)
    t1, t2 = t1 + ascc.initial_guess(o, v, hole, particle)[0], t2 + ascc.initial_guess(o, v, hole, particle)[1]
    t1so, t2so = closed_shell_to_so(t1, t2)
    E, r1so, r2so = BruteForce(hbar, _eri(Bbar), o, v).projections(t1so, t2so)
    R1, R2 = so_to_closed_shell(r1so, r2so, o, v)
    r1, r2 = cs_ccsd.residual(Bbar, fbar, t1, t2)
    assert np.abs(r1 - R1).max() < 1e-11
    assert np.abs(r2 - R2).max() < 1e-11
    e_ref = ascc.reference_energy(Bbar, fbar, o)
    assert abs(E - e_ref - cs_ccsd.energy(Bbar, fbar, t1, t2)) < 1e-11


@pytest.mark.parametrize("v,Q,seed,particle", [(3, 6, 41, 1), (4, 8, 42, 2), (5, 9, 43, 1)])
def test_two_electron_ascc_solution_is_an_eigenstate(v, Q, seed, particle):
    """With two electrons T1 + T2 is the full cluster operator, so a converged ASCC solution of Hbar is
    an exact eigenstate of H (Sec. II.A: FCI in the limit of a complete T): its energy is in the
    spectrum of H, and it is not the ground state the plain CC iteration would find."""
    o, hole = 1, 0
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    Bbar, fbar = ascc.transformed_inputs(B, eps, o, hole, particle)
    t1, t2 = ascc.initial_guess(o, v, hole, particle)
    res = solver.solve(lambda a, b: cs_ccsd.residual(Bbar, fbar, a, b),
                       lambda a, b: cs_ccsd.energy(Bbar, fbar, a, b), eps, t1, t2, maxiter=300, tol_rnorm=1e-11)
    assert res["converged"]
    E = ascc.reference_energy(Bbar, fbar, o) + res["E"]
    h = cs_ccsd.core_hamiltonian_df(B, np.diag(eps), o)
    H = BruteForce(h, _eri(B), o, v).hamiltonian_matrix()
    ev = np.linalg.eigvalsh(H)
    assert np.abs(ev - E).min() < 1e-9
    assert abs(E - ev.min()) > 1e-3


# ---- the second ansatz (Sec. II.D)

@pytest.mark.parametrize("alpha", [0.0, 0.15, -0.2])
@pytest.mark.parametrize("o,v,hole,particle", [(1, 3, 0, 1), (2, 3, 1, 2), (2, 2, 0, 3)])
def test_both_ansatz_give_the_reference_with_an_aufbau_part(o, v, hole, particle, alpha):
    """With gamma = -beta^2/2, e^{-S^dagger} e^{T^P(0)} |phi_0> = beta (alpha |phi_0> + S |phi_0>) for
    beta = 1/(1 + alpha); with S -> -S (the hole sign flipped) and beta = 1/(1 - alpha) the same state
    up to normalisation: both ansatz target alpha |phi_0> + S |phi_0> (Eq. (eqn:ref-with-nz-aufbau))."""
    B, eps = make_system(o, v, 4, 40, sigma=0.3)
    h = cs_ccsd.core_hamiltonian_df(B, np.diag(eps), o)
    bf = BruteForce(h, _eri(B), o, v)
    S, Sd = _s_ops(bf, o, v, hole, particle)
    target = alpha * bf.ref + S @ bf.ref
    b_plus, b_minus = ascc.two_ansatz_betas(alpha)
    for sign, beta in ((1.0, b_plus), (-1.0, b_minus)):
        t1, t2 = ascc.initial_guess(o, v, hole, particle, beta=sign * beta, gamma=-0.5 * beta * beta)
        t1so, t2so = closed_shell_to_so(t1, t2)
        psi = sla.expm(-sign * Sd) @ bf.exp_T(t1so, t2so, bf.ref)
        # psi = c * target for one scalar c
        c = (target @ psi) / (target @ target)
        assert np.abs(psi - c * target).max() < 1e-12
        assert abs(c - sign * beta) < 1e-12


def test_flipped_sign_is_the_transform_of_the_sign_flipped_orbitals():
    """S -> -S on H is the standard transform of H with the hole orbital's sign flipped (F B F, F h F),
    conjugated back by F: the two ansatz differ only by that phase convention."""
    o, v, Q, seed, hole, particle = 2, 3, 8, 32, 1, 3
    B, eps = make_system(o, v, Q, seed, sigma=0.3)
    h = cs_ccsd.core_hamiltonian_df(B, np.diag(eps), o)
    F = np.eye(o + v)
    F[hole, hole] = -1.0
    Bm, hm = ascc.transform(B, h, hole, particle, sign=-1.0)
    Bf, hf = ascc.transform(np.einsum("pr,Qrs,sq->Qpq", F, B, F), F @ h @ F, hole, particle, sign=1.0)
    assert np.abs(np.einsum("pr,Qrs,sq->Qpq", F, Bf, F) - Bm).max() < 1e-14
    assert np.abs(F @ hf @ F - hm).max() < 1e-14
    # and the flipped transform is the definition with -S
    bf = BruteForce(h, _eri(B), o, v)
    _, Sd = _s_ops(bf, o, v, hole, particle)
    Hdef = sla.expm(-Sd) @ bf.hamiltonian_matrix() @ sla.expm(Sd)
    assert np.abs(BruteForce(hm, _eri(Bm), o, v).hamiltonian_matrix() - Hdef).max() < 1e-12


def test_flipped_solve_equals_the_solve_on_sign_flipped_orbitals():
    o, v, Q, seed, hole, particle = 3, 12, 36, 7, 2, 3
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    F = np.ones(o + v)
    F[hole] = -1.0
    BF = B * F[None, :, None] * F[None, None, :]
    beta = ascc.two_ansatz_betas(0.1)[1]
    a = ascc.solve_state(B, eps, o, hole, particle, beta=beta, sign=-1.0)
    b = ascc.solve_state(BF, eps, o, hole, particle, beta=beta, sign=1.0)
    assert a["converged"] and b["converged"]
    assert abs(a["E"] - b["E"]) < 1e-9


@pytest.mark.parametrize("alpha", [0.0, 0.1])
def test_two_electron_two_ansatz_energies_are_eigenvalues(alpha):
    o, v, Q, seed, hole, particle = 1, 4, 8, 42, 0, 3
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    r = ascc.two_ansatz(B, eps, o, hole, particle, alpha, tol_rnorm=1e-11)
    assert r["converged"]
    h = cs_ccsd.core_hamiltonian_df(B, np.diag(eps), o)
    ev = np.linalg.eigvalsh(BruteForce(h, _eri(B), o, v).hamiltonian_matrix())
    for key in ("plus", "minus"):
        assert np.abs(ev - r[key]["E"]).min() < 1e-9
        assert r[key]["E"] - ev.min() > 1e-3
    assert r["E"] == pytest.approx(0.5 * (r["plus"]["E"] + r["minus"]["E"]))


def test_two_ansatz_keeps_the_single_converged_solution():
    """Sec. III.A: when one of the two solves fails, its partner's energy is reported alone."""
    o, v, Q, seed, hole, particle = 3, 12, 36, 7, 2, 3
    B, eps = make_system(o, v, Q, seed, sigma=converging_sigma(v, Q))
    full = ascc.two_ansatz(B, eps, o, hole, particle, 0.1)
    n_plus, n_minus = full["plus"]["iterations"], full["minus"]["iterations"]
    assert full["converged"] and n_plus != n_minus
    cap = min(n_plus, n_minus)  # only the faster solve finishes
    r = ascc.two_ansatz(B, eps, o, hole, particle, 0.1, maxiter=cap)
    faster = "plus" if n_plus < n_minus else "minus"
    assert r["any_converged"] and not r["converged"]
    assert r["used"] == (1 if faster == "plus" else 2)
    assert r["E"] == r[faster]["E"]
    none = ascc.two_ansatz(B, eps, o, hole, particle, 0.1, maxiter=3)
    assert not none["any_converged"] and none["used"] == 0
