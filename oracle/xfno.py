"""Extrapolated FNO (XFNO) on top of the oracle's truncation, CCSDT and EOM
(test infrastructure).

Part of the CPU oracle (tests, smoke check and CPU baseline only; no code
shared with the GPU library).  The paper (Computational Details) reports as
its M3 values FNO-EOM-CCSDT energies extrapolated from truncations at the
occupation thresholds 99.9%, 99.75% and 99.5%; the extrapolation formula is
in its supplement, which is not available.  Reading used here: every total
energy is fitted by a least-squares straight line in OCCT and the line is
evaluated at OCCT = 1 (no truncation).

Parity unpinned for the extrapolated values: no number of the paper fixes
them.  The fit itself is pinned by closed forms (exactly linear data, two
points, constant data) and each threshold's energies by the oracle's FNO,
CCSDT and EOM pins.
"""
from __future__ import annotations

import numpy as np

from . import cc, fno


def line_at(x, y, x0=1.0):
    """Value at x0 of the least-squares straight line through the points (x_i, y_i)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape != y.shape or x.size < 2:
        raise ValueError("need at least two points")
    mx, my = x.mean(), y.mean()
    slope = np.sum((x - mx) * (y - my)) / np.sum((x - mx) ** 2)
    return float(my + slope * (x0 - mx))


def xfno(fock, eri, nocc, occts, kind=None, nroots=0, e_nuc=0.0):
    """FNO-CCSDT (and, with ``kind``, the lowest ``nroots`` EOM target states by
    the oracle's Davidson) at each threshold, and the extrapolation of each
    total energy to OCCT = 1."""
    points = []
    for x in occts:
        tr = fno.truncate(fock, eri, nocc, occt=x)
        res = cc.solve_ccsdt(tr["fock"], tr["eri"], nocc, e_nuc=e_nuc)
        p = dict(occt=float(x), kept=int(tr["nvir"]), e_cc=float(res["e_tot"]),
                 e_mp2_trunc=float(fno.mp2_energy(tr["fock"], tr["eri"], nocc)))
        if kind:
            d = cc.davidson(tr["fock"], tr["eri"], nocc, res["amps"], kind, nroots, e_tol=1e-11, r_tol=1e-8)
            p["e_eom"] = res["e_tot"] + np.real(np.asarray(d["omega"][:nroots]))
        points.append(p)
    out = dict(points=points, e_cc_x=line_at(occts, [p["e_cc"] for p in points]))
    if kind:
        out["e_eom_x"] = np.array([line_at(occts, [p["e_eom"][r] for p in points]) for r in range(nroots)])
    return out
