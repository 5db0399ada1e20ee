"""The 1-CSF mixed triples T^M_3' of the excited-state ansatz, FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What (paper Sec. II.B.1, the projections of Eq. (eqn:H1TP) and the ansatz that follows them).  In
a 1-CSF state the only doubles amplitude of T^P(0) with all four indices primary is t_{h h}^{p p}
(closed shell; in spin orbitals t_{h_up h_dn}^{p_up p_dn}).  One contraction of the two-electron
part of the transformed Hamiltonian with it leaves a triple excitation that still holds at least
three of the four primary spin orbitals {h_up, h_dn, p_up, p_dn}: the determinants
phi_{h hbar k}^{p b c} (both hole spin orbitals emptied) and phi_{h j k}^{p pbar c} (both particle
spin orbitals filled).  That slice, of size O(o^2 v + o v^2), is T^M_3', and the excited-state
cluster operator is T = T1 + T2 + T^M_3'.  The ground state keeps T1 + T2.

Reading (the paper prints no working equations for these amplitudes).  The amplitudes are found
from the projections of Eq. (eqn:amp) onto every single, every double and every slice triple,
with T3 zero outside the slice; the energy is Eq. (eqn:energy), which T3 does not reach for a
two-body Hamiltonian.  The slice keeps only determinants with the reference's S_z.  Amplitudes
and residuals of the triples are spin-orbital: t_ijk^abc antisymmetric in (i, j, k) and in
(a, b, c), T3 = 1/36 sum t_ijk^abc a^dagger_a a^dagger_b a^dagger_c a_k a_j a_i, the convention
of ``oracle.bruteforce``.  Singles and doubles stay closed-shell (the alpha and alpha-beta
projections).

Working equations.  T1 enters by the T1 transform of ``oracle.cs_ccsd`` (Hhat = e^{-T1} Hbar
e^{T1}, exact, since T1 commutes with T2 and T3).  With the spin-orbital Fock matrix f and the
antisymmetrised integrals g_pqrs = <pq||rs> of Hhat (p, q created, r, s annihilated), the parts
of the projections that involve T3, and the whole triples projection, are the connected products
of Hhat with T2, T3, T2^2/2 and T2 T3 that have the right excitation rank:

  R1_ia     += 1/4 sum_mnef g_mnef t_imn^aef
  R2_ijab   += A2[ 1/4 sum_me f_me t_ijm^abe - 1/4 sum_mef g_amef t_ijm^efb - 1/4 sum_mne g_mnei t_mnj^eab ]
  R3_ijkabc  = A3[ - 1/4 g_abek t_ij^ec + 1/4 g_amjk t_im^bc                              (T2)
                   + 1/2 g_amef t_mi^eb t_jk^fc - 1/8 g_amef t_ij^ef t_mk^bc
                   - 1/8 g_mnek t_mn^ab t_ij^ec + 1/2 g_mnek t_mi^ea t_nj^bc
                   + 1/4 f_me t_mi^ab t_jk^ec                                             (T2 T2)
                   + 1/12 f_ae t_ijk^ebc - 1/12 f_mi t_mjk^abc + 1/24 g_abef t_ijk^efc
                   + 1/24 g_mnij t_mnk^abc - 1/4 g_amei t_mjk^ebc                          (T3)
                   - 1/8 g_mnef t_ij^ea t_mnk^fbc - 1/8 g_mnef t_mi^ab t_njk^efc
                   + 1/4 g_mnef t_mi^ea t_njk^fbc + 1/48 g_mnef t_ij^ef t_mnk^abc
                   + 1/48 g_mnef t_mn^ab t_ijk^efc - 1/24 g_mnef t_mi^ef t_njk^abc
                   - 1/24 g_mnef t_mn^ea t_ijk^fbc ]                                      (T2 T3)

summed over repeated indices, where A2 (A3) is the sum over the 4 (36) signed permutations of the
occupied and of the virtual labels of the output.  Each bracketed product is one connected
contraction pattern; as the antisymmetriser is applied to the plain product, a term's factor is
the usual one (1/2 per pair of equivalent lines, 1/2 of e^T for T2^2) divided by the number of
A's permutations that leave the product unchanged.  Every factor and sign is checked against the
brute-force projections of ``oracle.bruteforce`` (tests/test_oracle_triples.py), with generic
non-symmetric integrals, at sizes where no two of the patterns coincide.

No factorisation and no restriction of the sums to the slice: the full triples tensors are
formed, which limits this module to tiny systems (it is a checker).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import cs_ccsd
from .ascc import initial_guess, reference_energy, transformed_inputs
from .bruteforce import closed_shell_to_so, so_maps, so_to_closed_shell
from .so_ccsd import so_fock_and_antisym
from .solver import DIIS


def _signed_perms(n: int):
    out = []
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for x in range(n) for y in range(x + 1, n) if perm[x] > perm[y])
        out.append((perm, -1.0 if inv % 2 else 1.0))
    return out


def antisym3(x: np.ndarray) -> np.ndarray:
    """A3: the sum over the signed permutations of axes (0, 1, 2) and of axes (3, 4, 5)."""
    out = np.zeros_like(x)
    for po, so in _signed_perms(3):
        for pv, sv in _signed_perms(3):
            out += so * sv * x.transpose(*po, *(3 + q for q in pv))
    return out


def antisym2(x: np.ndarray) -> np.ndarray:
    """A2: the sum over the signed permutations of axes (0, 1) and of axes (2, 3)."""
    return x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)


def primary_spin_orbitals(no: int, nv: int, hole: int, particle: int):
    """The occupied spin orbitals (h_up, h_dn) and virtual ones (p_up, p_dn), in the occupied and
    virtual numbering of ``oracle.bruteforce`` (``particle`` is a full orbital index)."""
    a = particle - no
    if not (0 <= hole < no and 0 <= a < nv):
        raise ValueError("hole must be occupied and particle virtual")
    return (hole, no + hole), (a, nv + a)


def in_slice(occ, vir, no: int, nv: int, hole: int, particle: int) -> bool:
    """Whether the triple (occupied spin orbitals ``occ``, virtual ``vir``) belongs to T^M_3':
    at least three of the four primary spin orbitals, and the reference's S_z."""
    ph, pp = primary_spin_orbitals(no, nv, hole, particle)
    n_primary = sum(1 for i in occ if i in ph) + sum(1 for a in vir if a in pp)
    occ_alpha = sum(1 for i in occ if i < no)
    vir_alpha = sum(1 for a in vir if a < nv)
    return n_primary >= 3 and occ_alpha == vir_alpha


def slice_triples(no: int, nv: int, hole: int, particle: int):
    """The slice as a list of canonical triples (i < j < k, a < b < c) of spin-orbital indices."""
    out = []
    for occ in itertools.combinations(range(2 * no), 3):
        for vir in itertools.combinations(range(2 * nv), 3):
            if in_slice(occ, vir, no, nv, hole, particle):
                out.append(occ + vir)
    return out


def _orderings(triples, no: int, nv: int):
    """Flat indices into the [2no]^3 x [2nv]^3 tensor of the 36 orderings of every triple, and signs."""
    shape = (2 * no,) * 3 + (2 * nv,) * 3
    perms = [(po, pv, so * sv) for po, so in _signed_perms(3) for pv, sv in _signed_perms(3)]
    idx = np.zeros((len(triples), len(perms)), dtype=np.int64)
    sgn = np.zeros(len(perms))
    for n, t in enumerate(triples):
        for m, (po, pv, s) in enumerate(perms):
            idx[n, m] = np.ravel_multi_index(tuple(t[q] for q in po) + tuple(t[3 + q] for q in pv), shape)
            sgn[m] = s
    return idx, sgn


def slice_mask(no: int, nv: int, hole: int, particle: int) -> np.ndarray:
    """Boolean full tensor [2no]^3 x [2nv]^3, True on every ordering of every slice triple."""
    m = np.zeros((2 * no,) * 3 + (2 * nv,) * 3, dtype=bool)
    idx, _ = _orderings(slice_triples(no, nv, hole, particle), no, nv)
    m.flat[idx.ravel()] = True
    return m


def pack(t3: np.ndarray, triples) -> np.ndarray:
    """Unique amplitudes, one per canonical triple."""
    return np.array([t3[t] for t in triples])


def unpack(x: np.ndarray, triples, no: int, nv: int) -> np.ndarray:
    """Full antisymmetric tensor from the unique amplitudes (zero off the listed triples)."""
    t3 = np.zeros((2 * no,) * 3 + (2 * nv,) * 3)
    if len(triples):
        idx, sgn = _orderings(triples, no, nv)
        t3.flat[idx.ravel()] = (np.asarray(x)[:, None] * sgn[None, :]).ravel()
    return t3


def t3_terms(f: np.ndarray, g: np.ndarray, t2: np.ndarray, t3: np.ndarray, nocc: int):
    """The spin-orbital parts of the projections listed in the module docstring: (R1 from T3,
    R2 from T3, the whole R3), for f, g of the T1-transformed Hamiltonian and antisymmetric t2, t3."""
    o, v = slice(0, nocc), slice(nocc, None)
    def e(spec, *ops):
        return np.einsum(spec, *ops, optimize=True)

    goovv, gvovv, goovo = g[o, o, v, v], g[v, o, v, v], g[o, o, v, o]
    r1 = 0.25 * e("mnef,imnaef->ia", goovv, t3)
    r2 = antisym2(0.25 * e("me,ijmabe->ijab", f[o, v], t3) - 0.25 * e("amef,ijmefb->ijab", gvovv, t3)
                  - 0.25 * e("mnei,mnjeab->ijab", goovo, t3))
    x = -0.25 * e("abek,ijec->ijkabc", g[v, v, v, o], t2) + 0.25 * e("amjk,imbc->ijkabc", g[v, o, o, o], t2)
    x += 0.5 * e("amef,mieb,jkfc->ijkabc", gvovv, t2, t2) - 0.125 * e("amef,ijef,mkbc->ijkabc", gvovv, t2, t2)
    x += -0.125 * e("mnek,mnab,ijec->ijkabc", goovo, t2, t2) + 0.5 * e("mnek,miea,njbc->ijkabc", goovo, t2, t2)
    x += 0.25 * e("me,miab,jkec->ijkabc", f[o, v], t2, t2)
    x += e("ae,ijkebc->ijkabc", f[v, v], t3) / 12.0 - e("mi,mjkabc->ijkabc", f[o, o], t3) / 12.0
    x += e("abef,ijkefc->ijkabc", g[v, v, v, v], t3) / 24.0 + e("mnij,mnkabc->ijkabc", g[o, o, o, o], t3) / 24.0
    x += -0.25 * e("amei,mjkebc->ijkabc", g[v, o, v, o], t3)
    x += -0.125 * e("mnef,ijea,mnkfbc->ijkabc", goovv, t2, t3) - 0.125 * e("mnef,miab,njkefc->ijkabc", goovv, t2, t3)
    x += 0.25 * e("mnef,miea,njkfbc->ijkabc", goovv, t2, t3)
    x += e("mnef,ijef,mnkabc->ijkabc", goovv, t2, t3) / 48.0 + e("mnef,mnab,ijkefc->ijkabc", goovv, t2, t3) / 48.0
    x += -e("mnef,mief,njkabc->ijkabc", goovv, t2, t3) / 24.0 - e("mnef,mnea,ijkfbc->ijkabc", goovv, t2, t3) / 24.0
    return r1, r2, antisym3(x)


def residual(B: np.ndarray, fock: np.ndarray, t1: np.ndarray, t2: np.ndarray, t3: np.ndarray, mask: np.ndarray):
    """(r1, r2, r3): closed-shell singles and doubles residuals with the T3 couplings added, and the
    spin-orbital triples residual on ``mask`` (zero elsewhere), for the Hamiltonian given by B and
    its reference Fock matrix ``fock`` (Hbar's when called with the transformed inputs)."""
    no, nv = t1.shape
    r1, r2 = cs_ccsd.residual(B, fock, t1, t2)
    h = cs_ccsd.core_hamiltonian_df(B, fock, no)
    Bh, _, Fh = cs_ccsd.dressed(B, h, t1)
    f, g = so_fock_and_antisym(Fh, np.einsum("Qpq,Qrs->pqrs", Bh, Bh), no, nv)
    _, t2so = closed_shell_to_so(np.zeros_like(t1), t2)
    a1, a2, r3 = t3_terms(f, g, t2so, t3, 2 * no)
    c1, c2 = so_to_closed_shell(a1, a2, no, nv)
    return r1 + c1, r2 + c2, np.where(mask, r3, 0.0)


def denominators3(eps: np.ndarray, no: int) -> np.ndarray:
    """D_ijk^abc = e_i + e_j + e_k - e_a - e_b - e_c over spin orbitals (spatial orbital energies)."""
    nv = eps.shape[0] - no
    spatial, _ = so_maps(no, nv)
    eo = eps[spatial[:2 * no]]
    ev = eps[spatial[2 * no:]]
    d = eo[:, None, None] + eo[None, :, None] + eo[None, None, :]
    dv = ev[:, None, None] + ev[None, :, None] + ev[None, None, :]
    return d[:, :, :, None, None, None] - dv[None, None, None, :, :, :]


def solve_state(B, fock, no, hole, particle, beta=1.0, sign=1.0, tol_rnorm=1e-10, maxiter=400, diis_size=8):
    """ASCCSD (T1 + T2 + T^M_3') total energy of a 1-CSF state, solved from T^P(0) = beta S + gamma S^2
    (gamma = -beta^2/2, T3 = 0) by Jacobi steps t += R / D with DIIS over the vector (t1, t2, unique
    slice amplitudes); the same reading of Sec. III.B as ``oracle.solver``, with the slice appended."""
    from .solver import denominators

    f = np.diag(fock) if fock.ndim == 1 else fock
    eps = np.diag(f).copy()
    nv = B.shape[1] - no
    Bbar, fbar = transformed_inputs(B, f, no, hole, particle, sign)
    t1, t2 = initial_guess(no, nv, hole, particle, beta=sign * beta, gamma=-0.5 * beta * beta)
    triples = slice_triples(no, nv, hole, particle)
    mask = slice_mask(no, nv, hole, particle)
    d1, d2 = denominators(eps, no)
    idx, sgn = _orderings(triples, no, nv)

    def expand(x):
        t3 = np.zeros((2 * no,) * 3 + (2 * nv,) * 3)
        t3.flat[idx.ravel()] = (x[:, None] * sgn[None, :]).ravel()
        return t3

    d3 = denominators3(eps, no).flat[idx[:, 0]]
    x3 = np.zeros(len(triples))
    n1, n2 = t1.size, t2.size
    diis = DIIS(diis_size)
    hist = []
    converged = False
    for it in range(maxiter):
        r1, r2, r3 = residual(Bbar, fbar, t1, t2, expand(x3), mask)
        r3u = r3.flat[idx[:, 0]]
        e = cs_ccsd.energy(Bbar, fbar, t1, t2)
        rnorm = float(np.sqrt(np.sum(r1 * r1) + np.sum(r2 * r2) + np.sum(r3u * r3u)))
        hist.append(dict(it=it, E=e, rnorm=rnorm))
        if not np.isfinite(rnorm):
            break
        if rnorm <= tol_rnorm:
            converged = True
            break
        s1, s2, s3 = r1 / d1, r2 / d2, r3u / d3
        t1, t2, x3 = t1 + s1, t2 + s2, x3 + s3
        if it >= 1:
            diis.push(np.concatenate([t1.ravel(), t2.ravel(), x3]), np.concatenate([s1.ravel(), s2.ravel(), s3]))
            xv, _ = diis.extrapolate()
            if xv is not None:
                t1 = xv[:n1].reshape(t1.shape)
                t2 = xv[n1:n1 + n2].reshape(t2.shape)
                x3 = xv[n1 + n2:].copy()
    return dict(E=reference_energy(Bbar, fbar, no) + hist[-1]["E"], converged=converged, t1=t1, t2=t2,
                t3=expand(x3), triples=triples, iterations=len(hist), Bbar=Bbar, fbar=fbar)
