"""The PLASCC oracle (oracle/plascc.py) pinned on the CPU:

* against brute-force determinant projections of e^{-T} Hbar e^{T}, with T^M taken in the
  spin-orbital basis from the paper's definition (an amplitude with both primary and non-primary
  spin orbitals; Sec. II.B, Eq. (eqn: pnm split)) and the terms with two powers of it read off as
  the lam^2 coefficient of the projections at T2 = T2^R + lam T2^M (Sec. II.C);
* the degree-two structure of the doubles projection in T2 and the degree-one structure of the
  singles and the energy (no term of either carries two powers of T^M);
* reductions: no mixed amplitudes -> the CCSD residual; only mixed amplitudes and T1 = 0 -> a
  doubles equation linear in T2;
* size consistency (Sec. II.C: only connected terms are removed): the converged ground-state
  energy of two non-interacting fragments, primaries in one of them, is PLASCC of that fragment
  plus CCSD of the other.
"""
import numpy as np
import pytest

from gen.synth_df import make_system, random_amplitudes
from oracle import ascc, cs_ccsd, plascc, solver
from oracle.bruteforce import BruteForce, closed_shell_to_so, so_to_closed_shell


def _eri(B):
    return np.einsum("Qpq,Qrs->pqrs", B, B)


def _so_mixed_mask(no, nv, hole, particle):
    """[2o][2o][2v][2v]: spin-orbital doubles with both primary and non-primary spin orbitals."""
    occ_spatial = np.array([i % no for i in range(2 * no)])  # alpha block, then beta
    vir_spatial = np.array([no + (a % nv) for a in range(2 * nv)])
    po = occ_spatial == hole
    pv = vir_spatial == particle
    I, J, A, B = np.ix_(range(2 * no), range(2 * no), range(2 * nv), range(2 * nv))
    nprim = po[I].astype(int) + po[J] + pv[A] + pv[B]
    return (nprim > 0) & (nprim < 4)


CASES = [(2, 3, 8, 51, 1, 2), (2, 3, 7, 52, 0, 4), (3, 2, 6, 53, 2, 3), (2, 4, 9, 54, 0, 3)]


@pytest.mark.parametrize("transformed", [True, False])
@pytest.mark.parametrize("o,v,Q,seed,hole,particle", CASES)
def test_plascc_equals_brute_force_removal(o, v, Q, seed, hole, particle, transformed):
    B, eps = make_system(o, v, Q, seed, sigma=0.3)
    if transformed:  # the 1-CSF Hbar of the same hole and particle
        Bx, fx = ascc.transformed_inputs(B, eps, o, hole, particle)
    else:  # the ground state with the same term removal
        Bx, fx = B, np.diag(eps)
    h = cs_ccsd.core_hamiltonian_df(Bx, fx, o)
    bf = BruteForce(h, _eri(Bx), o, v)
    t1, t2 = random_amplitudes(o, v, seed + 5, 0.15, 0.15)
    g1, g2 = ascc.initial_guess(o, v, hole, particle)
    t1, t2 = t1 + g1, t2 + g2
    t1so, t2so = closed_shell_to_so(t1, t2)
    mso = _so_mixed_mask(o, v, hole, particle)
    tMso = np.where(mso, t2so, 0.0)
    tRso = t2so - tMso
    proj = {lam: bf.projections(t1so, tRso + lam * tMso) for lam in (-1.0, 0.0, 1.0, 2.0)}
    E = {k: p[0] for k, p in proj.items()}
    R1 = {k: p[1] for k, p in proj.items()}
    R2 = {k: p[2] for k, p in proj.items()}
    c = 0.5 * (R2[1.0] + R2[-1.0]) - R2[0.0]
    b = 0.5 * (R2[1.0] - R2[-1.0])
    # degree two in T2: the projection at lam = 2 follows from a, b, c
    assert np.abs(R2[2.0] - (R2[0.0] + 2 * b + 4 * c)).max() < 1e-11
    # singles and energy have no lam^2 part
    assert np.abs(R1[1.0] + R1[-1.0] - 2 * R1[0.0]).max() < 1e-11
    assert abs(E[1.0] + E[-1.0] - 2 * E[0.0]) < 1e-11
    assert np.abs(c).max() > 1e-4  # the removal is not empty
    r1_bf, r2_bf = so_to_closed_shell(R1[1.0], R2[1.0] - c, o, v)
    r1, r2 = plascc.residual(Bx, fx, t1, t2, hole, particle)
    assert np.abs(r1 - r1_bf).max() < 1e-11
    assert np.abs(r2 - r2_bf).max() < 1e-11
    e_ref = ascc.reference_energy(Bx, fx, o)
    assert abs(E[1.0] - e_ref - plascc.energy(Bx, fx, t1, t2)) < 1e-11


def test_mixed_mask_counts_and_the_spin_orbital_mask():
    o, v, hole, particle = 4, 6, 1, 7
    m = plascc.mixed_mask(o, v, hole, particle)
    # every amplitude except the non-primary ones ((o-1)^2 (v-1)^2) and the one all-primary one
    assert m.sum() == o * o * v * v - (o - 1) ** 2 * (v - 1) ** 2 - 1
    assert not m[hole, hole, particle - o, particle - o]
    # the closed-shell mask, mapped to spin orbitals, is the spin-orbital definition on every
    # nonzero spin-orbital amplitude
    t1, t2 = random_amplitudes(o, v, 3, 0.1, 0.1)
    _, tM = plascc.split(t2, hole, particle)
    _, tMso = closed_shell_to_so(np.zeros_like(t1), tM)
    _, t2so = closed_shell_to_so(np.zeros_like(t1), t2)
    assert np.abs(tMso - np.where(_so_mixed_mask(o, v, hole, particle), t2so, 0.0)).max() < 1e-15


def test_no_mixed_amplitudes_is_ccsd():
    o, v, Q, hole, particle = 3, 5, 10, 0, 5
    B, eps = make_system(o, v, Q, 61, sigma=0.2)
    t1, t2 = random_amplitudes(o, v, 62, 0.1, 0.1)
    t2 = np.where(plascc.mixed_mask(o, v, hole, particle), 0.0, t2)
    r1, r2 = plascc.residual(B, np.diag(eps), t1, t2, hole, particle)
    c1, c2 = cs_ccsd.residual(B, np.diag(eps), t1, t2)
    assert np.array_equal(r1, c1)
    assert np.abs(r2 - c2).max() < 1e-15


def test_only_mixed_amplitudes_gives_a_linear_doubles_equation():
    o, v, Q, hole, particle = 3, 5, 10, 2, 4
    B, eps = make_system(o, v, Q, 63, sigma=0.2)
    _, t2 = random_amplitudes(o, v, 64, 0.1, 0.2)
    _, tM = plascc.split(t2, hole, particle)
    z1 = np.zeros((o, v))
    f = np.diag(eps)
    R = [plascc.residual(B, f, z1, k * tM, hole, particle)[1] for k in (0.0, 1.0, 2.0)]
    assert np.abs(R[2] - 2 * R[1] + R[0]).max() < 1e-13
    full = [cs_ccsd.residual(B, f, z1, k * tM)[1] for k in (0.0, 1.0, 2.0)]
    assert np.abs(full[2] - 2 * full[1] + full[0]).max() > 1e-4  # CCSD is not linear there


def test_size_consistency_over_fragments():
    """Ground state with the term removal, primaries in fragment A: E(A+B) = E_PL(A) + E_CCSD(B)."""
    oa, va, qa = 2, 5, 9
    ob, vb, qb = 3, 4, 8
    Ba, ea = make_system(oa, va, qa, 71, sigma=0.15)
    Bb, eb = make_system(ob, vb, qb, 72, sigma=0.15)
    o, v, Q = oa + ob, va + vb, qa + qb
    n = o + v
    ia = list(range(oa)) + list(range(o, o + va))  # union order: occ A, occ B, vir A, vir B
    ib = list(range(oa, o)) + list(range(o + va, n))
    B = np.zeros((Q, n, n))
    B[np.ix_(range(qa), ia, ia)] = Ba
    B[np.ix_(range(qa, Q), ib, ib)] = Bb
    eps = np.zeros(n)
    eps[ia] = ea
    eps[ib] = eb
    hole_a, particle_a = 1, oa + 2  # in fragment A's own numbering

    def solve(Bx, ex, ox, prim):
        vx = ex.size - ox
        f = np.diag(ex)
        if prim is None:
            rf = lambda a, b: cs_ccsd.residual(Bx, f, a, b)  # noqa: E731
        else:
            rf = lambda a, b: plascc.residual(Bx, f, a, b, *prim)  # noqa: E731
        r = solver.solve(rf, lambda a, b: plascc.energy(Bx, f, a, b), ex, np.zeros((ox, vx)),
                         np.zeros((ox, ox, vx, vx)), maxiter=300, tol_rnorm=1e-11)
        assert r["converged"]
        return r["E"]

    e_union = solve(B, eps, o, (hole_a, o + (particle_a - oa)))
    e_a = solve(Ba, ea, oa, (hole_a, particle_a))
    e_b = solve(Bb, eb, ob, None)
    assert e_union == pytest.approx(e_a + e_b, abs=1e-10)
    # and the removal matters: plain CCSD of A differs
    assert abs(solve(Ba, ea, oa, None) - e_a) > 1e-7
