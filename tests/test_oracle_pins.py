"""The oracle pinned to things other than itself (CPU only).

* the definition: brute-force projections of e^{-T} H e^{T}|phi_0> (paper Eqs. (eqn:energy),
  (eqn:amp)) against the spin-orbital factorisation;
* the spin-adaptation relations (Supporting Information S1) tying the spin-orbital and the
  closed-shell residuals;
* first-order amplitudes / MP2 (Sec. II.B, Eqs. (eqn: perb doubles));
* the FCI limit for two electrons (Sec. II.A: CC recovers FCI with the full cluster operator);
* permutational symmetry of the density-fitted integrals; size extensivity (Sec. II.A);
  orbital invariance of the ground-state theory under occupied-occupied and virtual-virtual
  rotations (Sec. II.B); the pair symmetry of the closed-shell residual; a zero residual at
  convergence.
"""
import numpy as np
import pytest

from gen.synth_df import make_system, random_amplitudes, random_orthogonal, random_symmetric_fock
from oracle import cs_ccsd, solver
from oracle.bruteforce import BruteForce, closed_shell_to_so, core_hamiltonian, so_to_closed_shell
from oracle.so_ccsd import so_energy, so_fock_and_antisym, so_residual


def _eri(B):
    return np.einsum("Qpq,Qrs->pqrs", B, B)


CASES = [(1, 2, 4, 3, False), (2, 3, 8, 5, False), (2, 3, 8, 6, True), (3, 4, 10, 7, True), (2, 5, 9, 8, True)]


@pytest.mark.parametrize("o,v,Q,seed,full", CASES)
def test_spin_orbital_equations_equal_projection(o, v, Q, seed, full):
    B, eps = make_system(o, v, Q, seed, sigma=0.3)
    eri = _eri(B)
    fock = random_symmetric_fock(eps, 0.05, seed) if full else np.diag(eps)
    t1, t2 = random_amplitudes(o, v, seed + 50, 0.1, 0.1)
    t1so, t2so = closed_shell_to_so(t1, t2)
    bf = BruteForce(core_hamiltonian(eri, fock, o), eri, o, v)
    E, r1, r2 = bf.projections(t1so, t2so)
    e_ref = sum(core_hamiltonian(eri, fock, o)[i, i] + fock[i, i] for i in range(o))
    f, g = so_fock_and_antisym(fock, eri, o, v)
    R1, R2 = so_residual(f, g, t1so, t2so, 2 * o)
    assert abs(E - e_ref - so_energy(f, g, t1so, t2so, 2 * o)) < 1e-12
    assert np.abs(r1 - R1).max() < 1e-12
    assert np.abs(r2 - R2).max() < 1e-12


def test_projection_of_a_planted_mistake_is_caught():
    """A dropped term in the spin-orbital equations must show up against the projection."""
    o, v, Q, seed = 2, 3, 8, 5
    B, eps = make_system(o, v, Q, seed, sigma=0.3)
    eri = _eri(B)
    fock = np.diag(eps)
    t1, t2 = random_amplitudes(o, v, seed + 50, 0.1, 0.1)
    t1so, t2so = closed_shell_to_so(t1, t2)
    _, r1, r2 = BruteForce(core_hamiltonian(eri, fock, o), eri, o, v).projections(t1so, t2so)
    f, g = so_fock_and_antisym(fock, eri, o, v)
    R1, R2 = so_residual(f, g, t1so, t2so, 2 * o)
    # drop the quadratic tau part of the particle-particle ladder: W_abef without its tau term
    oo, vv = slice(0, 2 * o), slice(2 * o, None)
    tau = t2so + np.einsum("ia,jb->ijab", t1so, t1so) - np.einsum("ib,ja->ijab", t1so, t1so)
    missing = 0.5 * np.einsum("ijef,abef->ijab", tau, 0.25 * np.einsum("mnab,mnef->abef", tau, g[oo, oo, vv, vv]))
    assert np.abs(r2 - (R2 - missing)).max() > 1e-6


@pytest.mark.parametrize("o,v,Q,seed,full", CASES)
def test_closed_shell_equals_spin_orbital(o, v, Q, seed, full):
    B, eps = make_system(o, v, Q, seed, sigma=0.3)
    eri = _eri(B)
    fock = random_symmetric_fock(eps, 0.05, seed) if full else np.diag(eps)
    t1, t2 = random_amplitudes(o, v, seed + 50, 0.1, 0.1)
    t1so, t2so = closed_shell_to_so(t1, t2)
    f, g = so_fock_and_antisym(fock, eri, o, v)
    R1, R2 = so_residual(f, g, t1so, t2so, 2 * o)
    c1, c2 = so_to_closed_shell(R1, R2, o, v)
    r1, r2 = cs_ccsd.residual(B, fock, t1, t2)
    assert np.abs(r1 - c1).max() < 1e-12
    assert np.abs(r2 - c2).max() < 1e-12
    assert abs(cs_ccsd.energy(B, fock, t1, t2) - so_energy(f, g, t1so, t2so, 2 * o)) < 1e-12
    # the other spin blocks of the spin-orbital residual follow from the unique ones (S1)
    R1b = R1[o:, v:]
    assert np.abs(R1b - c1).max() < 1e-12
    Raa = R2[:o, :o, :v, :v]
    assert np.abs(Raa - (c2 - c2.transpose(1, 0, 2, 3))).max() < 1e-12


def test_first_jacobi_step_is_mp2():
    o, v, Q = 4, 12, 30
    B, eps = make_system(o, v, Q, 3)
    fock = np.diag(eps)
    z1, z2 = np.zeros((o, v)), np.zeros((o, o, v, v))
    r1, r2 = cs_ccsd.residual(B, fock, z1, z2)
    d1, d2 = solver.denominators(eps, o)
    t2 = r2 / d2
    g = np.einsum("Qia,Qjb->iajb", B[:, :o, o:], B[:, :o, o:])
    D = eps[:o, None, None, None] + eps[None, None, :o, None] - eps[None, o:, None, None] - eps[None, None, None, o:]
    # first-order doubles: t_ij^ab = (ia|jb) / D_ij^ab; singles vanish for a canonical HF Fock matrix
    assert np.abs(t2 - (g / D).transpose(0, 2, 1, 3)).max() < 1e-14
    assert np.abs(r1).max() < 1e-15
    e1 = cs_ccsd.energy(B, fock, z1, t2)
    assert e1 == pytest.approx(cs_ccsd.mp2_energy(B, eps, o), rel=1e-12)
    # the same through the oracle solver's second iteration
    res = solver.solve(lambda a, b: cs_ccsd.residual(B, fock, a, b), lambda a, b: cs_ccsd.energy(B, fock, a, b),
                       eps, z1, z2, maxiter=2, tol_rnorm=0.0)
    assert res["history"][1]["E"] == pytest.approx(cs_ccsd.mp2_energy(B, eps, o), rel=1e-12)


@pytest.mark.parametrize("v,seed", [(3, 1), (5, 2), (6, 3)])
def test_two_electron_ccsd_is_fci(v, seed):
    o, Q = 1, 6
    B, eps = make_system(o, v, Q, seed, sigma=0.15)
    eri = _eri(B)
    fock = np.diag(eps)
    res = solver.solve(lambda a, b: cs_ccsd.residual(B, fock, a, b), lambda a, b: cs_ccsd.energy(B, fock, a, b),
                       eps, np.zeros((o, v)), np.zeros((o, o, v, v)), maxiter=200, tol_rnorm=1e-12)
    assert res["converged"]
    h = core_hamiltonian(eri, fock, o)
    bf = BruteForce(h, eri, o, v)
    H = bf.hamiltonian_matrix()
    S2 = bf.s_squared_matrix()
    w, U = np.linalg.eigh(H)
    s2 = np.einsum("ik,ij,jk->k", U, S2, U)
    singlet = w[np.abs(s2) < 1e-8]
    e_ref = h[0, 0] + fock[0, 0]
    assert e_ref + res["E"] == pytest.approx(singlet.min(), abs=1e-10)


def test_integral_eightfold_symmetry():
    B, _ = make_system(3, 5, 7, 9)
    g = _eri(B)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0), (1, 0, 3, 2), (2, 3, 1, 0), (3, 2, 0, 1)]:
        assert np.array_equal(g, g.transpose(perm)) or np.abs(g - g.transpose(perm)).max() < 1e-15


def test_size_extensivity():
    """Two non-interacting closed-shell fragments: E_corr(A+B) = E_corr(A) + E_corr(B)."""
    oa, va, qa = 2, 5, 9
    ob, vb, qb = 3, 4, 8
    Ba, ea = make_system(oa, va, qa, 21, sigma=0.15)
    Bb, eb = make_system(ob, vb, qb, 22, sigma=0.15)
    o, v, Q = oa + ob, va + vb, qa + qb
    n = o + v
    # orbital order of the union: occupied of A, occupied of B, virtual of A, virtual of B
    ia = list(range(oa)) + list(range(o, o + va))
    ib = list(range(oa, o)) + list(range(o + va, n))
    B = np.zeros((Q, n, n))
    B[np.ix_(range(qa), ia, ia)] = Ba
    B[np.ix_(range(qa, Q), ib, ib)] = Bb
    eps = np.zeros(n)
    eps[ia] = ea
    eps[ib] = eb

    def solve(Bx, ex, ox):
        vx = ex.size - ox
        f = np.diag(ex)
        r = solver.solve(lambda a, b: cs_ccsd.residual(Bx, f, a, b), lambda a, b: cs_ccsd.energy(Bx, f, a, b),
                         ex, np.zeros((ox, vx)), np.zeros((ox, ox, vx, vx)), maxiter=200, tol_rnorm=1e-11)
        assert r["converged"]
        return r["E"]

    assert solve(B, eps, o) == pytest.approx(solve(Ba, ea, oa) + solve(Bb, eb, ob), abs=1e-10)


def test_orbital_rotation_invariance():
    """Occupied-occupied and virtual-virtual rotations leave the converged energy unchanged."""
    o, v, Q = 3, 8, 20
    B, eps = make_system(o, v, Q, 31, sigma=0.1)
    rng = np.random.default_rng(4)
    U = np.zeros((o + v, o + v))
    U[:o, :o] = random_orthogonal(o, rng)
    U[o:, o:] = random_orthogonal(v, rng)
    Br = np.einsum("pr,Qrs,qs->Qpq", U.T, B, U.T)
    f = np.diag(eps)
    fr = U.T @ f @ U

    def solve(Bx, fx):
        r = solver.solve(lambda a, b: cs_ccsd.residual(Bx, fx, a, b), lambda a, b: cs_ccsd.energy(Bx, fx, a, b),
                         np.diag(fx), np.zeros((o, v)), np.zeros((o, o, v, v)), maxiter=300, tol_rnorm=1e-11)
        assert r["converged"]
        return r["E"]

    assert np.abs(fr[:o, :o] - np.diag(np.diag(fr[:o, :o]))).max() > 1e-3  # really non-canonical
    assert solve(Br, fr) == pytest.approx(solve(B, f), abs=1e-9)


def test_residual_pair_symmetry_and_zero_at_convergence():
    o, v, Q = 5, 20, 60
    B, eps = make_system(o, v, Q, 0)
    f = np.diag(eps)
    t1, t2 = random_amplitudes(o, v, 3, 0.02, 0.02)
    r1, r2 = cs_ccsd.residual(B, f, t1, t2)
    assert np.abs(r2 - r2.transpose(1, 0, 3, 2)).max() < 1e-14
    res = solver.solve(lambda a, b: cs_ccsd.residual(B, f, a, b), lambda a, b: cs_ccsd.energy(B, f, a, b),
                       eps, np.zeros((o, v)), np.zeros((o, o, v, v)), maxiter=60, tol_rnorm=1e-8)
    assert res["converged"] and res["history"][-1]["rnorm"] <= 1e-8
    r1, r2 = cs_ccsd.residual(B, f, res["t1"], res["t2"])
    assert np.sqrt((r1 ** 2).sum() + (r2 ** 2).sum()) <= 1e-8


def test_diis_bordered_solve_matches_library_solve():
    rng = np.random.default_rng(0)
    E = rng.normal(size=(5, 40))
    Bm = E @ E.T
    c = solver.solve_bordered(Bm)
    A = np.zeros((6, 6))
    A[:5, :5] = Bm
    A[:5, 5] = A[5, :5] = -1
    rhs = np.zeros(6)
    rhs[5] = -1
    assert np.abs(c - np.linalg.solve(A, rhs)[:5]).max() < 1e-12
    assert abs(c.sum() - 1.0) < 1e-12
    # a singular system (repeated error vector) is refused
    E[4] = E[3]
    assert solver.solve_bordered(E @ E.T) is None


def test_jacobi_diis_reaches_the_exact_solution_of_a_linear_problem():
    """On a linear residual R(t) = b + A t with A = -diag(D) + E (E a small symmetric coupling, D the
    orbital-energy denominators), the diagonal-Jacobian step t <- t + R/D with DIIS must converge to
    the exact fixed point -A^-1 b (library solve) and in fewer iterations than the plain step."""
    rng = np.random.default_rng(7)
    o, v = 1, 3
    eps = np.concatenate([[-1.1], np.sort(rng.uniform(0.2, 2.0, v))])
    d1, d2 = solver.denominators(eps, o)
    d = np.concatenate([d1.ravel(), d2.ravel()])
    n = d.size
    E = rng.normal(size=(n, n))
    E = 0.25 * (E + E.T) * np.sqrt(np.outer(np.abs(d), np.abs(d))) / np.sqrt(n)
    A = -np.diag(d) + E
    b = rng.normal(size=n)
    x_exact = -np.linalg.solve(A, b)

    def residual(t1, t2):
        x = np.concatenate([t1.ravel(), t2.ravel()])
        r = b + A @ x
        return r[:o * v].reshape(o, v), r[o * v:].reshape(o, o, v, v)

    z1, z2 = np.zeros((o, v)), np.zeros((o, o, v, v))
    with_diis = solver.solve(residual, lambda a, c: 0.0, eps, z1, z2, maxiter=400, tol_rnorm=1e-13)
    plain = solver.solve(residual, lambda a, c: 0.0, eps, z1, z2, maxiter=400, tol_rnorm=1e-13, diis_size=1)
    for res in (with_diis, plain):
        assert res["converged"]
        x = np.concatenate([res["t1"].ravel(), res["t2"].ravel()])
        assert np.abs(x - x_exact).max() <= 1e-10 * (1 + np.abs(x_exact).max())
    assert len(with_diis["history"]) < len(plain["history"])


def test_convergence_tests_flip_at_the_known_iteration():
    """The solver's convergence test (Sec. III.A: max|R| and |dE| per iteration, plus the residual
    2-norm) on a problem whose iterates are known exactly: o = v = 1, eps = (-1/2, 1/2), so D1 = -1 and
    D2 = -2, and R(t) = -D t / 2, so every Jacobi step halves t (DIIS off).  From t = 1 the k-th
    iterate is t = 2^-k with r1 = 2^-(k+1), r2 = 2^-k (max|R| = 2^-k) and, for E = t1 + t2, dE = -2^(1-k).
    A tolerance equal to an achieved value separates <= from <, the negative dE catches a missing
    absolute value, and a pair of tests must both hold."""
    eps = np.array([-0.5, 0.5])
    d1, d2 = solver.denominators(eps, 1)
    assert d1.item() == -1.0 and d2.item() == -2.0

    def residual(t1, t2):
        return -0.5 * d1 * t1, -0.5 * d2 * t2

    def energy(t1, t2):
        return float(t1.sum() + t2.sum())

    one1, one2 = np.ones((1, 1)), np.ones((1, 1, 1, 1))

    def stop(**tol):
        res = solver.solve(residual, energy, eps, one1, one2, maxiter=40, diis_size=1, **tol)
        assert res["converged"]
        k = res["iterations"] - 1
        assert res["t1"].item() == 2.0 ** -k and res["t2"].item() == 2.0 ** -k  # the amplitudes tested
        return k

    assert stop(tol_rnorm=None, tol_rmax=2.0 ** -5) == 5       # max|R| <= tol, equality passes
    assert stop(tol_rnorm=None, tol_de=2.0 ** -4) == 6         # |dE| < tol, equality does not
    assert stop(tol_rnorm=float(np.sqrt(2.0 ** -8 + 2.0 ** -6))) == 3
    assert stop(tol_rnorm=None, tol_rmax=2.0 ** -5, tol_de=2.0 ** -2) == 5  # both must hold
    assert stop(tol_rnorm=None, tol_rmax=2.0 ** -2, tol_de=2.0 ** -4) == 6
    # the first iteration has no energy change: the energy test alone cannot pass there
    assert stop(tol_rnorm=None, tol_de=10.0) == 1
    hist = solver.solve(residual, energy, eps, one1, one2, maxiter=4, diis_size=1, tol_rnorm=None,
                        tol_rmax=1e-30)["history"]
    assert [h["dE"] for h in hist[1:]] == [-1.0, -0.5, -0.25]
    assert [h["rmax"] for h in hist] == [1.0, 0.5, 0.25, 0.125]
