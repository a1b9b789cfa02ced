"""Write sampled_elements.json: oracle values of randomly sampled residual and
sigma elements at the full-size workloads, for the GPU parity tests.

Run from the repository root: ``python tests/golden/make_sampled_elements.py``
(about 10 minutes on 8 cores).  Only the oracle computes values here; the
library is not imported.

* o=10, v_full=60 ground-state workload (seed 2), truncated by the oracle's
  FNO at OCCT 0.99: random T1, T2, T3 (numpy PCG64 seed 11, drawn in that
  order, N(0, 0.01), N(0, 0.01), N(0, 0.003) on the packed elements), the
  CCSDT residual (eq 5) at NSAMPLE random packed elements of each of R1, R2,
  R3 plus a few corner elements.
* o=12, v_full=80 workload (seed 3) truncated to 48 virtuals: random
  amplitudes and R vectors (PCG64 seed 17: T1, T2, T3, then one R block after
  another, N(0, 1) for R) and the EOM sigma of every variant (IP, EA, DIP,
  DEA) at NSAMPLE random packed elements of each block plus corners.

The sampled packed indices are drawn with PCG64 seed 99 per (workload,
block).  Each entry is [packed index, value].
"""
import json
import math
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import cc, fno, wick  # noqa: E402
from synthetic import config_hamiltonian  # noqa: E402
from tests.packing import LazyAntisym, colex_tuples  # noqa: E402

NSAMPLE = 256
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sampled_elements.json")


def pick(n, label):
    """NSAMPLE distinct random packed indices (all when fewer) plus the first and last."""
    rng = np.random.default_rng([99, sum(map(ord, label))])
    idx = rng.choice(n, size=min(NSAMPLE, n), replace=False).tolist()
    for c in (0, n - 1):
        if c not in idx:
            idx.append(c)
    return sorted(int(i) for i in idx)


def unravel(p, nocc, nvir, nh, np_):
    H = colex_tuples(nocc, nh) if nh else np.zeros((1, 0), np.int64)
    P = colex_tuples(nvir, np_) if np_ else np.zeros((1, 0), np.int64)
    h, q = divmod(p, len(P))
    return tuple(int(x) for x in H[h]) + tuple(int(x) for x in P[q])


# ---------------------------------------------------------------- workers
_G = {}


def _c2_setup():
    h = config_hamiltonian("C2")
    tr = fno.truncate(h.fock, h.eri, 10, occt=0.99)
    o, v = 10, tr["nvir"]
    rng = np.random.default_rng(11)
    t1 = rng.normal(0, 0.01, (o, v))
    t2p = rng.normal(0, 0.01, math.comb(o, 2) * math.comb(v, 2))
    t3p = rng.normal(0, 0.003, math.comb(o, 3) * math.comb(v, 3))
    amps = {1: t1, 2: LazyAntisym(t2p, o, v, 2, 2)[:, :, :, :], 3: LazyAntisym(t3p, o, v, 3, 3)}
    return tr, o, v, amps


def _c3_setup(kind):
    h = config_hamiltonian("C3")
    tr = fno.truncate(h.fock, h.eri, 12, nvir_keep=48)
    o, v = 12, 48
    rng = np.random.default_rng(17)
    t1 = rng.normal(0, 0.01, (o, v))
    t2p = rng.normal(0, 0.01, math.comb(o, 2) * math.comb(v, 2))
    t3p = rng.normal(0, 0.002, math.comb(o, 3) * math.comb(v, 3))
    _, blocks = wick.EOM_SPACES[kind]
    rvec = [rng.normal(0, 1.0, math.comb(o, b[0]) * math.comb(v, b[1])) for b in blocks]
    amps = {1: t1, 2: LazyAntisym(t2p, o, v, 2, 2)[:, :, :, :], 3: LazyAntisym(t3p, o, v, 3, 3)}
    rb = {b: (LazyAntisym(x, o, v, *b) if b[0] + b[1] == 6 else LazyAntisym(x, o, v, *b)[(slice(None),) * (b[0] + b[1])])
          for b, x in zip(blocks, rvec)}
    return tr, o, v, amps, blocks, rb


def work_c2(args):
    k, p = args
    if "C2" not in _G:
        _G["C2"] = _c2_setup()
    tr, o, v, amps = _G["C2"]
    idx = unravel(p, o, v, k, k)
    return float(cc.cc_residual_element(tr["fock"], tr["eri"], o, amps, k, idx))


def work_c3(args):
    kind, bi, p = args
    if kind not in _G:
        _G[kind] = _c3_setup(kind)
    tr, o, v, amps, blocks, rb = _G[kind]
    b = blocks[bi]
    idx = unravel(p, o, v, b[0], b[1])
    return float(cc.eom_sigma_element(tr["fock"], tr["eri"], o, amps, kind, rb, b, idx))


def main():
    out = {"nsample": NSAMPLE}
    with Pool(int(os.environ.get("GOLDEN_PROCS", "7"))) as pool:
        # ground state, o=10, v=59
        h = config_hamiltonian("C2")
        v = fno.truncate(h.fock, h.eri, 10, occt=0.99)["nvir"]
        o = 10
        c2 = {"nvir": v}
        for k in (1, 2, 3):
            n = math.comb(o, k) * math.comb(v, k)
            ps = pick(n, f"C2:R{k}")
            vals = pool.map(work_c2, [(k, p) for p in ps], chunksize=4)
            c2[f"R{k}"] = [[p, x] for p, x in zip(ps, vals)]
            print("C2", k, len(ps), flush=True)
        out["C2"] = c2
        # EOM sigma, o=12, v=48
        o, v = 12, 48
        c3 = {}
        for kind in ("IP", "EA", "DIP", "DEA"):
            _, blocks = wick.EOM_SPACES[kind]
            c3[kind] = {}
            for bi, b in enumerate(blocks):
                n = math.comb(o, b[0]) * math.comb(v, b[1])
                ps = pick(n, f"C3:{kind}:{bi}")
                vals = pool.map(work_c3, [(kind, bi, p) for p in ps], chunksize=2)
                c3[kind][f"{b[0]}h{b[1]}p"] = [[p, x] for p, x in zip(ps, vals)]
                print("C3", kind, b, len(ps), flush=True)
        out["C3"] = c3
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(OUT)


if __name__ == "__main__":
    main()
