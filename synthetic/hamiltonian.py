"""Seeded synthetic spin-orbital Hamiltonians (inputs only, no method arithmetic).

The paper's molecules need integrals, basis sets and geometries that are not
available, so every workload here is a synthetic stand-in of the same kind of
object the method consumes (Section 1.2, eqs 8-10): a spin-orbital Fock
matrix that is diagonal in the canonical orbitals, and antisymmetrized
two-electron integrals <pq||rs>.

Recipe (stated once, used by the oracle and the GPU library alike):

* ``rng = numpy.random.Generator(numpy.random.PCG64(seed))``; draw order is
  occupied energies, virtual energies, then the two-electron tensor.
* occupied orbital energies ~ U[eocc], virtual ~ U[evir], each sorted
  ascending; the Fock matrix is ``diag(eocc ++ evir)`` (so f_ov = 0).
* chemist-notation integrals (pq|rs): i.i.d. N(0, sigma^2) entries, averaged
  over the 8 real-orbital permutations (pq|rs)=(qp|rs)=(pq|sr)=(rs|pq)...
* <pq|rs> = (pr|qs) and <pq||rs> = <pq|rs> - <pq|sr>, stored as a dense
  n^4 row-major float64 array (occupied orbitals first).
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class SyntheticHamiltonian:
    nocc: int
    nvir: int
    fock: np.ndarray          # (n, n) float64
    eri: np.ndarray           # (n, n, n, n) float64, <pq||rs>
    e_nuc: float = 0.0
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nocc + self.nvir

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.fock).tobytes())
        h.update(np.ascontiguousarray(self.eri).tobytes())
        return h.hexdigest()


def make_hamiltonian(nocc: int, nvir: int, seed: int,
                     eocc=(-2.0, -0.5), evir=(0.3, 3.0), sigma: float = 0.05,
                     e_nuc: float = 0.0, decay: float = 0.0) -> SyntheticHamiltonian:
    """Draw one seeded Hamiltonian with ``nocc`` occupied and ``nvir`` virtual spin-orbitals.

    ``decay`` > 0 scales every integral <pq||rs> by w_p w_q w_r w_s with
    w = 1 on occupied orbitals and w = exp(-a / decay) on the a-th virtual (in
    ascending energy), so the higher virtuals couple more weakly and their MP2
    natural occupations fall off (as the diffuse functions of a real basis
    do); the permutational symmetries are kept exactly.
    """
    if nocc < 0 or nvir < 0:
        raise ValueError("nocc and nvir must be non-negative")
    n = nocc + nvir
    rng = np.random.Generator(np.random.PCG64(seed))
    eo = np.sort(rng.uniform(eocc[0], eocc[1], nocc))
    ev = np.sort(rng.uniform(evir[0], evir[1], nvir))
    g = rng.normal(0.0, sigma, size=(n, n, n, n))
    acc = g.copy()
    for perm in ((1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
                 (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)):
        acc += g.transpose(perm)
    del g
    acc *= 0.125
    phys = acc.transpose(0, 2, 1, 3)            # <pq|rs> = (pr|qs)
    eri = np.ascontiguousarray(phys - phys.transpose(0, 1, 3, 2))
    del acc, phys
    if decay > 0:
        w = np.concatenate([np.ones(nocc), np.exp(-np.arange(nvir) / decay)])
        eri *= np.einsum("p,q,r,s->pqrs", w, w, w, w)
    fock = np.diag(np.concatenate([eo, ev])).astype(np.float64)
    return SyntheticHamiltonian(nocc, nvir, fock, eri, e_nuc, seed,
                                dict(eocc=tuple(eocc), evir=tuple(evir), sigma=sigma, decay=decay))


def full_virtuals_for(v_kept: int) -> int:
    """Virtual count drawn before FNO truncation when a workload fixes the kept count.

    The 60 -> 36 ratio of the o=10 workload (5:3) is reused, rounded up.
    """
    return int(math.ceil(5 * v_kept / 3))


# Named workloads.  Sizes are spin-orbitals; "keep" fixes the FNO kept count,
# "occt" the cumulative-occupation threshold (None = no truncation).
CONFIGS = {
    "C1": dict(nocc=4, nvir=12, seed=1, evir=(0.3, 3.0), occt=None, keep=None),
    "C2": dict(nocc=10, nvir=60, seed=2, evir=(0.2, 6.0), occt=0.99, keep=None),
    "C3": dict(nocc=12, nvir=full_virtuals_for(48), seed=3, evir=(0.3, 3.0), occt=None, keep=48),
    "C5eval": dict(nocc=14, nvir=full_virtuals_for(56), seed=5, evir=(0.3, 3.0), occt=None, keep=56),
    "C5train": dict(nocc=8, nvir=full_virtuals_for(32), seed=1000, evir=(0.3, 3.0), occt=None, keep=32),
}


def config_hamiltonian(name: str, seed: int | None = None) -> SyntheticHamiltonian:
    c = CONFIGS[name]
    return make_hamiltonian(c["nocc"], c["nvir"], c["seed"] if seed is None else seed,
                            evir=c["evir"])


def batch_instance_shapes(count: int = 16, seed: int = 4):
    """(nocc, nvir_kept, seed) of the uneven-size batch: o ~ U{6..12}, v ~ U{24..48}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        o = int(rng.integers(6, 13))
        v = int(rng.integers(24, 49))
        out.append((o, v, 400 + k))
    return out
