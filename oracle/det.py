"""Determinant-space brute force (test infrastructure, CPU only).

This module is part of the oracle: a slow, literal evaluation of the
definitions the paper states, used only by tests, the smoke check and the
CPU baseline.  It shares no code with the GPU library.

* CC residual, eq (5):  r_mu = <Phi_mu| e^{-T} H e^{T} |Phi_0>  for any T.
* CC energy, eq (6):    E = <Phi_0| e^{-T} H e^{T} |Phi_0>.
* EOM, eqs (1)-(4):     H-bar = e^{-T} H e^{T} applied in the N-m / N+m
  electron sector to R|Phi_0>, projected on the R space.
* FCI: exact eigenvalues of H in each particle-number sector.

Conventions (spin-orbitals, occupied orbitals 0..o-1 first):
* H = sum_pq h_pq p^+ q + 1/4 sum_pqrs <pq||rs> p^+ q^+ s r with
  h_pq = f_pq - sum_i <pi||qi>, so that the given f is the Fock matrix of
  Phi_0 and E_ref = sum_i f_ii - 1/2 sum_ij <ij||ij>.
* Unique amplitude (holes h1<...<hk, particles p1<...<pl) labels the string
  tau = p1^+ ... pl^+ hk ... h1; <Phi_mu| = <0| tau^+.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np
import scipy.sparse as sp


def _parity(x: np.ndarray) -> np.ndarray:
    return (np.bitwise_count(x) & 1).astype(np.int8)


class Sector:
    """All determinants with ``nel`` electrons in ``n`` spin-orbitals (bit p = orbital p)."""

    def __init__(self, n: int, nel: int):
        self.n, self.nel = n, nel
        dets = [sum(1 << p for p in c) for c in itertools.combinations(range(n), nel)]
        self.dets = np.array(sorted(dets), dtype=np.uint64)

    @property
    def dim(self) -> int:
        return len(self.dets)

    def index(self, d: np.ndarray) -> np.ndarray:
        return np.searchsorted(self.dets, d)

    def apply(self, ops):
        """Apply the operator product ops[0] ops[1] ... (rightmost acts first).

        ops: sequence of (orbital, dagger).  Returns (new_dets, sign, valid).
        """
        d = self.dets.copy()
        sign = np.ones(len(d), dtype=np.int8)
        valid = np.ones(len(d), dtype=bool)
        for p, dag in reversed(ops):
            bit = np.uint64(1 << p)
            occ = (d & bit) != 0
            valid &= (~occ) if dag else occ
            sign = np.where(_parity(d & (bit - np.uint64(1))) == 1, -sign, sign)
            d = d ^ bit
        return d, sign, valid

    def operator(self, terms, target: "Sector | None" = None) -> sp.csr_matrix:
        """Sparse matrix of sum_k c_k * ops_k from this sector into ``target``."""
        target = target or self
        rows, cols, vals = [], [], []
        src = np.arange(self.dim)
        for c, ops in terms:
            if c == 0.0:
                continue
            d, s, ok = self.apply(ops)
            if not ok.any():
                continue
            rows.append(target.index(d[ok]))
            cols.append(src[ok])
            vals.append(c * s[ok].astype(np.float64))
        if not rows:
            return sp.csr_matrix((target.dim, self.dim))
        m = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(target.dim, self.dim))
        return m.tocsr()

    def det_of(self, occ_list) -> int:
        d = sum(1 << p for p in occ_list)
        i = int(self.index(np.array([d], dtype=np.uint64))[0])
        assert self.dets[i] == d
        return i


def core_hamiltonian(fock: np.ndarray, eri: np.ndarray, nocc: int) -> np.ndarray:
    """h_pq = f_pq - sum_i <pi||qi> (makes f the Fock matrix of Phi_0)."""
    return fock - np.einsum("piqi->pq", eri[:, :nocc, :, :nocc])


def reference_energy(fock, eri, nocc, e_nuc=0.0) -> float:
    o = slice(0, nocc)
    return float(np.trace(fock[o, o]) - 0.5 * np.einsum("ijij->", eri[o, o, o, o]) + e_nuc)


def hamiltonian_terms(fock, eri, nocc, tol=0.0):
    """H = sum h_pq p^+ q + sum_{p<q, r<s} <pq||rs> p^+ q^+ s r as (coef, ops) terms."""
    n = fock.shape[0]
    h = core_hamiltonian(fock, eri, nocc)
    terms = []
    for p in range(n):
        for q in range(n):
            if abs(h[p, q]) > tol:
                terms.append((h[p, q], ((p, 1), (q, 0))))
    for p, q in itertools.combinations(range(n), 2):
        for r, s in itertools.combinations(range(n), 2):
            c = eri[p, q, r, s]
            if abs(c) > tol:
                terms.append((c, ((p, 1), (q, 1), (s, 0), (r, 0))))
    return terms


def excitation_string(holes, parts):
    """tau = p1^+ ... pl^+ hk ... h1 as an ops tuple."""
    return tuple((p, 1) for p in parts) + tuple((h, 0) for h in reversed(holes))


def unique_labels(nocc: int, nvir: int, nh: int, np_: int):
    """Unique (holes, particles) labels, holes ascending then particles ascending."""
    occ = range(nocc)
    vir = range(nocc, nocc + nvir)
    return [(h, p) for h in itertools.combinations(occ, nh) for p in itertools.combinations(vir, np_)]


class DetModel:
    """Second-quantized model over n = nocc + nvir spin-orbitals."""

    def __init__(self, fock, eri, nocc, e_nuc=0.0):
        self.fock = np.asarray(fock, dtype=np.float64)
        self.eri = np.asarray(eri, dtype=np.float64)
        self.nocc = nocc
        self.n = self.fock.shape[0]
        self.nvir = self.n - nocc
        self.e_nuc = e_nuc
        self._sectors = {}
        self._H = {}
        self._hterms = hamiltonian_terms(self.fock, self.eri, nocc)

    def sector(self, nel) -> Sector:
        if nel not in self._sectors:
            self._sectors[nel] = Sector(self.n, nel)
        return self._sectors[nel]

    def H(self, nel) -> sp.csr_matrix:
        if nel not in self._H:
            s = self.sector(nel)
            self._H[nel] = s.operator(self._hterms) + self.e_nuc * sp.identity(s.dim, format="csr")
        return self._H[nel]

    def fci(self, nel, k=None) -> np.ndarray:
        """All (or the k lowest) eigenvalues of H in the nel-electron sector."""
        Hm = self.H(nel).toarray()
        w = np.linalg.eigvalsh(Hm)
        return w if k is None else w[:k]

    # ----- cluster operator as a matrix on any sector -----
    def T_operator(self, nel, amps) -> sp.csr_matrix:
        """amps: dict rank -> dense antisymmetric array t[h1..hk, p1..pk] (particle indices 0-based in the virtual space)."""
        s = self.sector(nel)
        terms = []
        o = self.nocc
        for k, t in amps.items():
            for holes, parts in unique_labels(self.nocc, self.nvir, k, k):
                c = t[tuple(holes) + tuple(p - o for p in parts)]
                if c != 0.0:
                    terms.append((c, excitation_string(holes, parts)))
        return s.operator(terms)

    @staticmethod
    def _expm_nilpotent(T, x, sign=1.0):
        out = x.copy()
        term = x.copy()
        for k in range(1, 64):
            term = (sign / k) * (T @ term)
            if not np.any(term):
                break
            out += term
        return out

    def similarity(self, nel, amps):
        """Return a function x -> e^{-T} H e^{T} x on the nel-electron sector."""
        T = self.T_operator(nel, amps)
        H = self.H(nel)

        def apply(x):
            y = self._expm_nilpotent(T, x, 1.0)
            y = H @ y
            return self._expm_nilpotent(T, y, -1.0)
        return apply

    def reference_vector(self):
        s = self.sector(self.nocc)
        x = np.zeros(s.dim)
        x[s.det_of(range(self.nocc))] = 1.0
        return x

    def _basis(self, nel, nh, np_):
        """Target-sector positions and signs of tau_mu |Phi_0> for the unique labels."""
        src = self.sector(self.nocc)
        dst = self.sector(nel)
        ref = src.det_of(range(self.nocc))
        idx, sgn = [], []
        labels = unique_labels(self.nocc, self.nvir, nh, np_)
        for holes, parts in labels:
            d = int(src.dets[ref])
            s = 1
            for p, dag in reversed(excitation_string(holes, parts)):
                below = d & ((1 << p) - 1)
                if bin(below).count("1") & 1:
                    s = -s
                d ^= (1 << p)
            i = int(dst.index(np.array([d], dtype=np.uint64))[0])
            assert int(dst.dets[i]) == d
            idx.append(i)
            sgn.append(s)
        return labels, np.array(idx, dtype=np.int64), np.array(sgn, dtype=np.float64)

    def cc_residual(self, amps, ranks=(1, 2, 3)):
        """Eq (5) projections for every unique label of each rank, plus eq (6) energy."""
        x = self.reference_vector()
        y = self.similarity(self.nocc, amps)(x)
        out = {}
        for k in ranks:
            labels, idx, sgn = self._basis(self.nocc, k, k)
            out[k] = (labels, y[idx] * sgn)
        ref = self.sector(self.nocc).det_of(range(self.nocc))
        return out, float(y[ref])

    def eom_space(self, kind):
        """(electron change, [(nh, np) blocks]) for the four variants (Section 1.1, eqs 3-4)."""
        return {
            "IP": (-1, [(1, 0), (2, 1), (3, 2)]),
            "DIP": (-2, [(2, 0), (3, 1), (4, 2)]),
            "EA": (+1, [(0, 1), (1, 2), (2, 3)]),
            "DEA": (+2, [(0, 2), (1, 3), (2, 4)]),
        }[kind]

    def R_operator(self, kind, rblocks):
        """R = sum_mu r_mu tau_mu as a sparse map from the N sector to the target sector.

        rblocks: dict (nh, np) -> dense antisymmetric array r[h..., p...].
        """
        dn, _ = self.eom_space(kind)
        src = self.sector(self.nocc)
        dst = self.sector(self.nocc + dn)
        o = self.nocc
        terms = []
        for (nh, np_), r in rblocks.items():
            for holes, parts in unique_labels(self.nocc, self.nvir, nh, np_):
                c = r[tuple(holes) + tuple(p - o for p in parts)]
                if c != 0.0:
                    terms.append((c, excitation_string(holes, parts)))
        return src.operator(terms, dst)

    def eom_sigma(self, kind, amps, rblocks):
        """sigma = P [H-bar, R] |Phi_0> for any T (the connected EOM sigma vector).

        [H-bar, R]|0> = H-bar R|0> - R H-bar|0>; its eigenvalues on the R space
        are E_target - E_CC.  Returns a list of (block, labels, values).
        """
        dn, allblocks = self.eom_space(kind)
        nel = self.nocc + dn
        Rop = self.R_operator(kind, rblocks)
        x0 = self.reference_vector()
        y = self.similarity(nel, amps)(Rop @ x0) - Rop @ self.similarity(self.nocc, amps)(x0)
        out = []
        for nh, np_ in allblocks:
            labels, idx, sgn = self._basis(nel, nh, np_)
            out.append(((nh, np_), labels, y[idx] * sgn if len(idx) else np.zeros(0)))
        return out

    def eom_matrix(self, kind, amps, e_cc, blocks=None):
        """Dense <Phi_mu| (H-bar - E_CC) |Phi_nu> over the R space of ``kind``.

        Returns (matrix, list of (block, labels)).
        """
        dn, allblocks = self.eom_space(kind)
        blocks = blocks or allblocks
        nel = self.nocc + dn
        app = self.similarity(nel, amps)
        dst = self.sector(nel)
        bases = [self._basis(nel, nh, np_) for nh, np_ in blocks]
        idx = np.concatenate([b[1] for b in bases])
        sgn = np.concatenate([b[2] for b in bases])
        dim = len(idx)
        M = np.zeros((dim, dim))
        for c in range(dim):
            x = np.zeros(dst.dim)
            x[idx[c]] = sgn[c]
            y = app(x)
            M[:, c] = y[idx] * sgn
        M -= e_cc * np.eye(dim)
        return M, [(blk, b[0]) for blk, b in zip(blocks, bases)]


# ----- dense <-> unique conversion helpers used by the oracle tests -----
def dense_from_unique(values, labels, nocc, nvir, nh, np_):
    """Scatter unique values into a dense fully antisymmetric array [holes..., particles...]."""
    shape = (nocc,) * nh + (nvir,) * np_
    out = np.zeros(shape)
    for val, (holes, parts) in zip(values, labels):
        pv = tuple(p - nocc for p in parts)
        for ph in itertools.permutations(range(nh)):
            sh = _perm_sign(ph)
            for pp in itertools.permutations(range(np_)):
                sp_ = _perm_sign(pp)
                out[tuple(holes[i] for i in ph) + tuple(pv[i] for i in pp)] = sh * sp_ * val
    return out


def unique_from_dense(arr, labels, nocc):
    return np.array([arr[tuple(h) + tuple(p - nocc for p in ps)] for h, ps in labels])


@lru_cache(maxsize=None)
def _perm_sign_cached(p):
    p = list(p)
    s = 1
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


def _perm_sign(p):
    return _perm_sign_cached(tuple(p))
