"""Frozen natural orbitals from the MP2 virtual density (test infrastructure).

Part of the CPU oracle (tests, smoke check and CPU baseline only; no code
shared with the GPU library).  Follows Section 1.2 step by step:

1. MP2 amplitudes t_ij^ab = <ab||ij> / e_ij^ab               (eq 8)
2. denominators  e_ij^ab = f_ii + f_jj - f_aa - f_bb            (eq 9)
3. virtual density D_ab = 1/2 sum_cij <cb||ij><ij||ca> / (e_ij^cb e_ij^ca)   (eq 10)
4. diagonalise D; natural orbitals sorted by descending occupation; keep the
   most occupied ones (truncation) and freeze the rest.
5. semicanonicalise the kept virtual block of the Fock matrix (optional in
   the paper; always done here) and transform f and <pq||rs>.

Readings where the paper is silent (listed in the design notes):
* truncation by cumulative occupation: keep the smallest k with
  sum_{l<=k} n_l >= occt * sum_l n_l (relative slack 1e-12); a degenerate
  group straddling the cut (|n_k - n_{k+1}| <= 1e-10 n_k) is kept whole;
  the alternative scheme keeps a fixed count ``nvir_keep``.
* semicanonical orbitals in ascending energy, each eigenvector's largest
  |component| made positive.
"""
from __future__ import annotations

import numpy as np


def mp2_denominators(fock, nocc):
    """e_ij^ab = f_ii + f_jj - f_aa - f_bb (eq 9)."""
    eo = np.diag(fock)[:nocc]
    ev = np.diag(fock)[nocc:]
    return eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]


def mp2_amplitudes(fock, eri, nocc):
    """t[i,j,a,b] = <ab||ij> / e_ij^ab (eq 8)."""
    o, v = slice(0, nocc), slice(nocc, fock.shape[0])
    return eri[v, v, o, o].transpose(2, 3, 0, 1) / mp2_denominators(fock, nocc)


def mp2_energy(fock, eri, nocc):
    """E_MP2 = 1/4 sum <ij||ab> t_ij^ab."""
    o, v = slice(0, nocc), slice(nocc, fock.shape[0])
    return 0.25 * float(np.einsum("ijab,ijab->", eri[o, o, v, v], mp2_amplitudes(fock, eri, nocc)))


def virtual_density(fock, eri, nocc):
    """D_ab of eq (10), written out term by term."""
    o, v = slice(0, nocc), slice(nocc, fock.shape[0])
    e = mp2_denominators(fock, nocc)           # e[i,j,a,b]
    num1 = eri[v, v, o, o]                     # <cb||ij> -> [c,b,i,j]
    num2 = eri[o, o, v, v]                     # <ij||ca> -> [i,j,c,a]
    # D_ab = 1/2 sum_{c,i,j} <cb||ij> <ij||ca> / (e_ij^{cb} e_ij^{ca})
    return 0.5 * np.einsum("cbij,ijca,ijcb,ijca->ab", num1, num2, 1.0 / e, 1.0 / e, optimize=True)


def occt_cut(occ, occt, tie_tol=1e-10):
    """Number of natural orbitals kept for a cumulative-occupation threshold."""
    occ = np.asarray(occ)
    nv = len(occ)
    if not (0.0 < occt <= 1.0):
        raise ValueError("occt must lie in (0, 1]")
    if occt == 1.0 or nv == 0:
        return nv
    total = occ.sum()
    csum = np.cumsum(occ)
    target = occt * total * (1.0 - 1e-12)
    k = int(np.searchsorted(csum, target) + 1)
    k = min(k, nv)
    while k < nv and abs(occ[k - 1] - occ[k]) <= tie_tol * abs(occ[k - 1]):
        k += 1
    return k


def _fix_signs(U):
    U = U.copy()
    for j in range(U.shape[1]):
        i = np.argmax(np.abs(U[:, j]))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    return U


def natural_orbitals(fock, eri, nocc):
    """Occupations (descending) and NO coefficients (columns) of the virtual density."""
    D = virtual_density(fock, eri, nocc)
    w, U = np.linalg.eigh(0.5 * (D + D.T))
    order = np.argsort(-w, kind="stable")
    return w[order], _fix_signs(U[:, order])


def truncate(fock, eri, nocc, occt=1.0, nvir_keep=0):
    """FNO truncation + semicanonicalisation; returns the transformed problem.

    Returns dict(fock, eri, nocc, nvir, occ, C) where C (v_full x v_kept)
    maps canonical virtuals to the kept semicanonical natural orbitals.
    """
    n = fock.shape[0]
    nv = n - nocc
    occ, U = natural_orbitals(fock, eri, nocc)
    k = int(nvir_keep) if nvir_keep and nvir_keep > 0 else occt_cut(occ, occt)
    if k > nv:
        raise ValueError("nvir_keep exceeds the virtual space")
    Uk = U[:, :k]
    fvv = Uk.T @ fock[nocc:, nocc:] @ Uk
    e, V = np.linalg.eigh(0.5 * (fvv + fvv.T))
    V = _fix_signs(V)
    C = Uk @ V
    full = np.zeros((n, nocc + k))
    full[:nocc, :nocc] = np.eye(nocc)
    full[nocc:, nocc:] = C
    f2 = full.T @ fock @ full
    g = eri
    for ax in range(4):
        g = np.tensordot(g, full, axes=([0], [0]))   # rotates axis 0 to the end
    return dict(fock=f2, eri=np.ascontiguousarray(g), nocc=nocc, nvir=k, occ=occ, C=C,
                e_mp2_full=mp2_energy(fock, eri, nocc))
