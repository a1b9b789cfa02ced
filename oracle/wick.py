"""Wick's-theorem evaluation of CC and EOM-CC matrix elements (test infrastructure).

Part of the CPU oracle; only tests, the smoke check and the CPU baseline use
it, and it shares no code with the GPU library.

What it computes, straight from the definitions:

* eq (5): r_mu(T) = <Phi_mu| e^{-T} H e^{T} |Phi_0> = <Phi_mu| (H_N e^T)_C |Phi_0>
  for mu a single, double or triple excitation, and eq (6) for the energy;
* eqs (1)-(4): the EOM sigma vector for the IP, DIP, EA and DEA operator
  spaces, sigma_mu = <Phi_mu| (H_N e^T R)_C |Phi_0>, whose eigenvalues are
  E_target - E_CC.

H_N = sum f_pq {p^+ q} + 1/4 sum <pq||rs> {p^+ q^+ s r} is the normal-ordered
Hamiltonian (f the Fock matrix).  Each operator product is expanded by
Wick's theorem for normal-ordered strings with respect to the Fermi vacuum
Phi_0: every full contraction between different strings is enumerated, its
sign is (-1)^(number of crossing contraction lines), and only products in
which H_N is connected to every cluster/EOM operator are kept.

Contractions that differ only by which slot of an antisymmetric group takes
which line give equal values (the sign of the permutation cancels the
antisymmetry of the tensor), so the enumeration keeps one representative per
"skeleton" (the multiset of lines between strings, external lines labelled)
and multiplies it by the number of contractions in the class.  No other
factorisation or reordering is done: each class is one ``numpy.einsum``.

Amplitude conventions: T_k = (1/k!)^2 sum t_{i1..ik}^{a1..ak} a1^+..ak^+ ik..i1,
R = 1/(h! p!) sum r_{i1..ih}^{a1..ap} a1^+..ap^+ ih..i1, all arrays dense and
antisymmetric within their hole group and within their particle group.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass
from functools import lru_cache

import numpy as np

OCC, VIR = "o", "v"


@dataclass(frozen=True)
class _Op:
    sid: int      # which string
    slot: int     # tensor slot of that string
    space: str    # OCC / VIR
    dag: bool     # creation (a^+) or annihilation (a) in the particle sense

    @property
    def q_annihilator(self) -> bool:
        return self.dag if self.space == OCC else not self.dag


@dataclass(frozen=True)
class _String:
    kind: str            # "bra", "f", "w", "t", "r"
    spaces: tuple        # tensor slot spaces
    ops: tuple           # (slot, space, dag) in operator order
    prefactor: float
    tag: tuple           # identity used when deciding whether two strings are interchangeable


def _bra(nh, np_):
    spaces = (OCC,) * nh + (VIR,) * np_
    ops = tuple((s, OCC, True) for s in range(nh)) + \
        tuple((nh + s, VIR, False) for s in reversed(range(np_)))
    return _String("bra", spaces, ops, 1.0, ("bra",))


def _fblock(s1, s2):
    return _String("f", (s1, s2), ((0, s1, True), (1, s2, False)), 1.0, ("f", s1, s2))


def _wblock(s1, s2, s3, s4):
    ops = ((0, s1, True), (1, s2, True), (3, s4, False), (2, s3, False))
    return _String("w", (s1, s2, s3, s4), ops, 0.25, ("w", s1, s2, s3, s4))


def _excitation(kind, nh, np_):
    spaces = (OCC,) * nh + (VIR,) * np_
    ops = tuple((nh + s, VIR, True) for s in range(np_)) + \
        tuple((s, OCC, False) for s in reversed(range(nh)))
    pref = 1.0 / (math.factorial(nh) * math.factorial(np_))
    return _String(kind, spaces, ops, pref, (kind, nh, np_))


def _hamiltonian_blocks():
    out = []
    for s in itertools.product((OCC, VIR), repeat=2):
        out.append(_fblock(*s))
    for s in itertools.product((OCC, VIR), repeat=4):
        out.append(_wblock(*s))
    return out


def _pairings(ops):
    """All full contractions of a flattened operator list (list of index pairs)."""
    n = len(ops)
    for sp in (OCC, VIR):
        qa = sum(1 for o in ops if o.space == sp and o.q_annihilator)
        qc = sum(1 for o in ops if o.space == sp and not o.q_annihilator)
        if qa != qc:
            return []
    used = [False] * n
    pairs = []
    out = []

    def rec():
        try:
            x = used.index(False)
        except ValueError:
            out.append(list(pairs))
            return
        ox = ops[x]
        if not ox.q_annihilator:
            return
        used[x] = True
        for y in range(x + 1, n):
            if used[y]:
                continue
            oy = ops[y]
            if oy.sid == ox.sid or oy.space != ox.space or oy.q_annihilator:
                continue
            used[y] = True
            pairs.append((x, y))
            rec()
            pairs.pop()
            used[y] = False
        used[x] = False

    rec()
    return out


def _crossings(pairs):
    c = 0
    for i in range(len(pairs)):
        a, b = pairs[i]
        for j in range(i + 1, len(pairs)):
            p, q = pairs[j]
            if (a < p < b < q) or (p < a < q < b):
                c += 1
    return c


@dataclass
class Term:
    """One contraction class: coef * prod_k tensor_k[letters_k] summed over dummies."""
    coef: float
    factors: tuple    # ((kind, tag, letters), ...) excluding the bra
    out: str          # external letters in bra slot order
    key: tuple = ()   # skeleton key (lines between strings, external lines labelled)

    def einsum_spec(self):
        return ",".join(f[2] for f in self.factors) + "->" + self.out


_LETTERS = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"


def _expand(strings):
    """All contraction classes of <bra| s1 s2 ... |0>, H_N (string 1) connected to all others."""
    ops = []
    for sid, s in enumerate(strings):
        for slot, space, dag in s.ops:
            ops.append(_Op(sid, slot, space, dag))
    classes = {}
    # permutations of interchangeable strings (same tag) among the strings after H
    groups = {}
    for sid, s in enumerate(strings):
        if sid >= 2:
            groups.setdefault(s.tag, []).append(sid)
    perms = [dict()]
    for tag, sids in groups.items():
        new = []
        for base in perms:
            for p in itertools.permutations(sids):
                d = dict(base)
                d.update(zip(sids, p))
                new.append(d)
        perms = new
    for pairing in _pairings(ops):
        touched = set()
        for x, y in pairing:
            a, b = ops[x].sid, ops[y].sid
            if a == 1:
                touched.add(b)
            if b == 1:
                touched.add(a)
        if any(sid not in touched for sid in range(2, len(strings))):
            continue
        sign = -1.0 if _crossings(pairing) & 1 else 1.0
        best = None
        for pm in perms:
            key = []
            for x, y in pairing:
                ox, oy = ops[x], ops[y]
                a = pm.get(ox.sid, ox.sid)
                b = pm.get(oy.sid, oy.sid)
                ext = ox.slot if ox.sid == 0 else -1
                key.append((a, b, ox.space, ext))
            key = tuple(sorted(key))
            if best is None or key < best:
                best = key
        if best in classes:
            classes[best][1] += 1
        else:
            classes[best] = [(pairing, sign), 1]
    terms = []
    bra = strings[0]
    for key, ((pairing, sign), count) in classes.items():
        letters = {}
        ext = {}
        nxt = len(bra.spaces)
        for x, y in pairing:
            ox, oy = ops[x], ops[y]
            if ox.sid == 0:
                L = _LETTERS[ox.slot]
                letters[(ox.sid, ox.slot)] = L
                letters[(oy.sid, oy.slot)] = L
                ext[ox.slot] = L
            else:
                L = _LETTERS[nxt]
                nxt += 1
                letters[(ox.sid, ox.slot)] = L
                letters[(oy.sid, oy.slot)] = L
        coef = sign * count
        factors = []
        for sid in range(1, len(strings)):
            s = strings[sid]
            coef *= s.prefactor
            lets = "".join(letters[(sid, k)] for k in range(len(s.spaces)))
            factors.append((s.kind, s.tag, lets))
        out = "".join(ext[k] for k in range(len(bra.spaces)))
        sig = tuple(st.tag for st in strings)
        terms.append(Term(coef, tuple(factors), out, (sig, key)))
    return terms


def _multisets(ranks, maxcount):
    for n in range(maxcount + 1):
        for combo in itertools.combinations_with_replacement(ranks, n):
            yield combo


@lru_cache(maxsize=None)
def cc_terms(k: int, t_ranks=(1, 2, 3)):
    """Contraction classes of <Phi_k| (H_N e^T)_C |Phi_0> (k=0 gives the correlation energy)."""
    bra = _bra(k, k)
    terms = []
    for combo in _multisets(t_ranks, 4):
        counts = {r: combo.count(r) for r in set(combo)}
        extra = 1.0
        for r, c in counts.items():
            extra /= math.factorial(c)
        ts = [_excitation("t", r, r) for r in combo]
        for H in _hamiltonian_blocks():
            for term in _expand([bra, H] + ts):
                term.coef *= extra
                terms.append(term)
    return tuple(terms)


EOM_SPACES = {
    # (electron change, R blocks (nh, np)) -- eqs (3)-(4) read with the ranks
    # stated in Section 1.1 and the conclusions (EA/DEA start at n = 0 holes).
    "IP": (-1, ((1, 0), (2, 1), (3, 2))),
    "DIP": (-2, ((2, 0), (3, 1), (4, 2))),
    "EA": (+1, ((0, 1), (1, 2), (2, 3))),
    "DEA": (+2, ((0, 2), (1, 3), (2, 4))),
}


@lru_cache(maxsize=None)
def eom_terms(mu: tuple, nu: tuple, t_ranks=(1, 2, 3)):
    """Contraction classes of <Phi_mu| (H_N e^T R_nu)_C |Phi_0> for blocks mu, nu = (nh, np)."""
    bra = _bra(*mu)
    r = _excitation("r", *nu)
    terms = []
    for combo in _multisets(t_ranks, 3):
        counts = {rk: combo.count(rk) for rk in set(combo)}
        extra = 1.0
        for rk, c in counts.items():
            extra /= math.factorial(c)
        ts = [_excitation("t", rk, rk) for rk in combo]
        for H in _hamiltonian_blocks():
            for term in _expand([bra, H, r] + ts):
                term.coef *= extra
                terms.append(term)
    return tuple(terms)


def merge_external(terms, nh, np_):
    """Keep one class per orbit under permutations of like external indices.

    The bra is antisymmetric in its hole labels and in its particle labels,
    so for G = S_nh x S_np and the antisymmetrizer A[X] = sum_g sgn(g) X o g,
    sum over an orbit O of classes = (|O| / |G|) A[X_rep].  Returns
    (terms, |G|); evaluate the merged list with ``antisymmetrize=True``.
    """
    groups = {}
    order = []
    for t in terms:
        sig, key = t.key
        best = None
        for ph in itertools.permutations(range(nh)):
            for pp in itertools.permutations(range(np_)):
                relabel = list(ph) + [nh + p for p in pp]
                k2 = tuple(sorted((a, b, sp, relabel[e] if e >= 0 else -1) for a, b, sp, e in key))
                if best is None or k2 < best:
                    best = k2
        okey = (sig, best)
        if okey not in groups:
            groups[okey] = [t, set()]
            order.append(okey)
        groups[okey][1].add(key)
    out = []
    for okey in order:
        rep, members = groups[okey]
        out.append(Term(rep.coef * len(members), rep.factors, rep.out, rep.key))
    return out, math.factorial(nh) * math.factorial(np_)


def antisymmetrize(x, nh, np_):
    """A[X] = sum over hole and particle permutations of sgn * X permuted."""
    out = np.zeros_like(x)
    for ph in itertools.permutations(range(nh)):
        sh = _sign(ph)
        for pp in itertools.permutations(range(np_)):
            perm = list(ph) + [nh + p for p in pp]
            out += (sh * _sign(pp)) * x.transpose(perm)
    return out


def _sign(p):
    p = list(p)
    s = 1
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


class Tensors:
    """Blocks of f and <pq||rs> plus amplitude arrays, looked up by term factor tags."""

    def __init__(self, fock, eri, nocc):
        self.fock = np.asarray(fock)
        self.eri = np.asarray(eri)
        self.nocc = nocc
        self._blocks = {}
        self.amps = {}

    def _sl(self, s):
        return slice(0, self.nocc) if s == OCC else slice(self.nocc, self.fock.shape[0])

    def get(self, kind, tag):
        if kind in ("f", "w"):
            if tag not in self._blocks:
                sl = tuple(self._sl(s) for s in tag[1:])
                src = self.fock if kind == "f" else self.eri
                self._blocks[tag] = np.ascontiguousarray(src[sl])
            return self._blocks[tag]
        return self.amps.get(tag)


def evaluate(terms, tensors: Tensors, shape, fixed=None):
    """Sum of all terms as a dense array over the external indices.

    ``fixed``: optional tuple of external index values; then a scalar is
    returned (one output element, computed without forming the full array).
    """
    out = 0.0 if fixed is not None else np.zeros(shape)
    for term in terms:
        ops = []
        skip = False
        for kind, tag, lets in term.factors:
            arr = tensors.get(kind, tag)
            if arr is None:
                skip = True
                break
            ops.append((arr, lets))
        if skip or term.coef == 0.0:
            continue
        if fixed is not None:
            sub = dict(zip(term.out, fixed))
            arrs, specs = [], []
            for arr, lets in ops:
                idx = tuple(sub.get(c, slice(None)) for c in lets)
                arrs.append(arr[idx])
                specs.append("".join(c for c in lets if c not in sub))
            val = np.einsum(",".join(specs) + "->", *arrs, optimize=True)
            out += term.coef * float(val)
        else:
            spec = ",".join(l for _, l in ops) + "->" + term.out
            out += term.coef * np.einsum(spec, *[a for a, _ in ops], optimize=True)
    return out
