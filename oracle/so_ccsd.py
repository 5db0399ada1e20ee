"""Spin-orbital CCSD residuals and energy (textbook factorisation), FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The residuals are the projections of Eq. (eqn:amp) (paper Sec. II.A) with T = T1 + T2 and S = 0,
written with the standard spin-orbital intermediates of Stanton, Gauss, Watts and Bartlett
(J. Chem. Phys. 94, 4334 (1991)), as tabulated in the Crawford-Schaefer review the paper cites
for coupled-cluster theory.  The residual is R = RHS - D t, with D_i^a = f_ii - f_aa and
D_ij^ab = f_ii + f_jj - f_aa - f_bb; the diagonal Fock elements enter only through D, so an
off-diagonal (non-canonical, non-HF) Fock matrix is handled exactly.

Pinned against ``oracle.bruteforce`` (the definition) on tiny inputs.
"""
from __future__ import annotations

import numpy as np

from .bruteforce import so_maps


def so_fock_and_antisym(fock: np.ndarray, eri: np.ndarray, no: int, nv: int):
    """Spin-orbital Fock f_PQ and antisymmetrised <PQ||RS> = (PR|QS) - (PS|QR) with spin deltas."""
    spatial, spin = so_maps(no, nv)
    same = (spin[:, None] == spin[None, :]).astype(float)
    f = fock[np.ix_(spatial, spatial)] * same
    chem = eri[np.ix_(spatial, spatial, spatial, spatial)] * same[:, :, None, None] * same[None, None, :, :]
    phys = chem.transpose(0, 2, 1, 3)
    return f, np.ascontiguousarray(phys - phys.transpose(0, 1, 3, 2))


def so_energy(f, g, t1, t2, nocc):
    """E_corr = sum f_ia t_i^a + 1/4 sum <ij||ab> t_ij^ab + 1/2 sum <ij||ab> t_i^a t_j^b."""
    o, v = slice(0, nocc), slice(nocc, None)
    e = np.einsum("ia,ia->", f[o, v], t1)
    e += 0.25 * np.einsum("ijab,ijab->", g[o, o, v, v], t2)
    e += 0.5 * np.einsum("ijab,ia,jb->", g[o, o, v, v], t1, t1)
    return float(e)


def so_residual(f, g, t1, t2, nocc):
    """Spin-orbital residuals (R1[i,a], R2[i,j,a,b]) = RHS - D*t."""
    o, v = slice(0, nocc), slice(nocc, None)
    fd = np.diag(f)
    nso = f.shape[0]
    nvir = nso - nocc
    Dia = fd[o][:, None] - fd[v][None, :]
    Dijab = fd[o][:, None, None, None] + fd[o][None, :, None, None] - fd[v][None, None, :, None] - fd[v][None, None, None, :]

    tau_t = t2 + 0.5 * (np.einsum("ia,jb->ijab", t1, t1) - np.einsum("ib,ja->ijab", t1, t1))
    tau = t2 + np.einsum("ia,jb->ijab", t1, t1) - np.einsum("ib,ja->ijab", t1, t1)

    fov = f[o, v]
    Fae = f[v, v] * (1.0 - np.eye(nvir))
    Fae -= 0.5 * np.einsum("me,ma->ae", fov, t1)
    Fae += np.einsum("mf,mafe->ae", t1, g[o, v, v, v])
    Fae -= 0.5 * np.einsum("mnaf,mnef->ae", tau_t, g[o, o, v, v])

    Fmi = f[o, o] * (1.0 - np.eye(nocc))
    Fmi += 0.5 * np.einsum("ie,me->mi", t1, fov)
    Fmi += np.einsum("ne,mnie->mi", t1, g[o, o, o, v])
    Fmi += 0.5 * np.einsum("inef,mnef->mi", tau_t, g[o, o, v, v])

    Fme = fov + np.einsum("nf,mnef->me", t1, g[o, o, v, v])

    Wmnij = g[o, o, o, o].copy()
    x = np.einsum("je,mnie->mnij", t1, g[o, o, o, v])
    Wmnij += x - x.transpose(0, 1, 3, 2)
    Wmnij += 0.25 * np.einsum("ijef,mnef->mnij", tau, g[o, o, v, v])

    Wabef = g[v, v, v, v].copy()
    x = np.einsum("mb,amef->abef", t1, g[v, o, v, v])
    Wabef -= x - x.transpose(1, 0, 2, 3)
    Wabef += 0.25 * np.einsum("mnab,mnef->abef", tau, g[o, o, v, v])

    Wmbej = g[o, v, v, o].copy()
    Wmbej += np.einsum("jf,mbef->mbej", t1, g[o, v, v, v])
    Wmbej -= np.einsum("nb,mnej->mbej", t1, g[o, o, v, o])
    Wmbej -= np.einsum("jnfb,mnef->mbej", 0.5 * t2 + np.einsum("jf,nb->jnfb", t1, t1), g[o, o, v, v])

    # singles right-hand side
    r1 = fov.copy()
    r1 += np.einsum("ie,ae->ia", t1, Fae)
    r1 -= np.einsum("ma,mi->ia", t1, Fmi)
    r1 += np.einsum("imae,me->ia", t2, Fme)
    r1 -= np.einsum("nf,naif->ia", t1, g[o, v, o, v])
    r1 -= 0.5 * np.einsum("imef,maef->ia", t2, g[o, v, v, v])
    r1 -= 0.5 * np.einsum("mnae,nmei->ia", t2, g[o, o, v, o])

    # doubles right-hand side
    r2 = g[o, o, v, v].copy()
    x = np.einsum("ijae,be->ijab", t2, Fae - 0.5 * np.einsum("mb,me->be", t1, Fme))
    r2 += x - x.transpose(0, 1, 3, 2)
    x = np.einsum("imab,mj->ijab", t2, Fmi + 0.5 * np.einsum("je,me->mj", t1, Fme))
    r2 -= x - x.transpose(1, 0, 2, 3)
    r2 += 0.5 * np.einsum("mnab,mnij->ijab", tau, Wmnij)
    r2 += 0.5 * np.einsum("ijef,abef->ijab", tau, Wabef)
    x = np.einsum("imae,mbej->ijab", t2, Wmbej) - np.einsum("ie,ma,mbej->ijab", t1, t1, g[o, v, v, o])
    r2 += x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)
    x = np.einsum("ie,abej->ijab", t1, g[v, v, v, o])
    r2 += x - x.transpose(1, 0, 2, 3)
    x = np.einsum("ma,mbij->ijab", t1, g[o, v, o, o])
    r2 -= x - x.transpose(0, 1, 3, 2)

    return r1 - Dia * t1, r2 - Dijab * t2
