"""Test-side conversions between dense antisymmetric arrays and the library's
packed layout (no method arithmetic).

Packed layout: each antisymmetric group stores strictly increasing tuples in
colexicographic order (tuple x0<..<x{g-1} at sum_t C(x_t, t+1)); the hole
group is the leading (slow) index, the particle group the trailing one.
"""
import itertools
import math

import numpy as np


def colex_tuples(n, g):
    combos = list(itertools.combinations(range(n), g))
    combos.sort(key=lambda t: t[::-1])
    return np.array(combos, dtype=np.int64).reshape(len(combos), g)


def pack(dense, nh, np_):
    """Dense [h..., p...] antisymmetric array -> packed vector."""
    nocc = dense.shape[0] if nh else 0
    nvir = dense.shape[-1] if np_ else 0
    H = colex_tuples(nocc, nh) if nh else np.zeros((1, 0), np.int64)
    P = colex_tuples(nvir, np_) if np_ else np.zeros((1, 0), np.int64)
    idx = tuple(H[:, k][:, None] for k in range(nh)) + tuple(P[:, k][None, :] for k in range(np_))
    return np.asarray(dense[idx]).reshape(-1)


def _binom_table(nmax, gmax):
    t = np.zeros((nmax + 1, gmax + 1), dtype=np.int64)
    for n in range(nmax + 1):
        for k in range(gmax + 1):
            t[n, k] = math.comb(n, k)
    return t


class LazyAntisym:
    """Dense view of a packed antisymmetric block, materialised slice by slice."""

    def __init__(self, packed, nocc, nvir, nh, np_):
        self.v = np.asarray(packed)
        self.nocc, self.nvir, self.nh, self.np_ = nocc, nvir, nh, np_
        self.shape = (nocc,) * nh + (nvir,) * np_
        self.ncp = math.comb(nvir, np_)
        self.B = _binom_table(max(nocc, nvir) + 1, max(nh, np_) + 1)

    def _rank(self, x):
        # x: (..., g) values; returns (rank, sign) with sign 0 on repeats
        g = x.shape[-1]
        sign = np.ones(x.shape[:-1], dtype=np.int64)
        for a in range(g):
            for b in range(a + 1, g):
                sign = np.where(x[..., a] > x[..., b], -sign, sign)
                sign = np.where(x[..., a] == x[..., b], 0, sign)
        xs = np.sort(x, axis=-1)
        r = np.zeros(x.shape[:-1], dtype=np.int64)
        for t in range(g):
            r += self.B[xs[..., t], t + 1]
        return r, sign

    def __getitem__(self, idx):
        if not isinstance(idx, tuple):
            idx = (idx,)
        idx = idx + (slice(None),) * (len(self.shape) - len(idx))
        axes = []
        for d, (k, n) in enumerate(zip(idx, self.shape)):
            axes.append(np.arange(n)[k] if isinstance(k, slice) else np.array([k]))
        grids = np.meshgrid(*axes, indexing="ij")
        hol = np.stack(grids[:self.nh], axis=-1) if self.nh else None
        par = np.stack(grids[self.nh:], axis=-1) if self.np_ else None
        rh, sh = self._rank(hol) if self.nh else (0, 1)
        rp, sp = self._rank(par) if self.np_ else (0, 1)
        s = sh * sp
        flat = rh * self.ncp + rp
        vals = np.where(s != 0, s * self.v[np.where(s != 0, flat, 0)], 0.0)
        keep = tuple(0 if not isinstance(k, slice) else slice(None) for k in idx)
        return vals[keep]


def unpack(packed, nocc, nvir, nh, np_):
    """Packed vector -> full dense antisymmetric array (small sizes)."""
    return LazyAntisym(packed, nocc, nvir, nh, np_)[(slice(None),) * (nh + np_)]


def unpack_fast(packed, nocc, nvir, nh, np_):
    """Packed vector -> dense antisymmetric array by scattering each signed permutation."""
    from itertools import permutations

    H = colex_tuples(nocc, nh)
    Pt = colex_tuples(nvir, np_)
    vals = np.asarray(packed).reshape(len(H), len(Pt))
    out = np.zeros((nocc,) * nh + (nvir,) * np_)

    def sgn(p):
        s, p = 1, list(p)
        for i in range(len(p)):
            while p[i] != i:
                j = p[i]
                p[i], p[j] = p[j], p[i]
                s = -s
        return s

    for ph in permutations(range(nh)):
        for pp in permutations(range(np_)):
            idx = tuple(H[:, k][:, None] for k in ph) + tuple(Pt[:, k][None, :] for k in pp)
            out[idx] = sgn(ph) * sgn(pp) * vals
    return out
