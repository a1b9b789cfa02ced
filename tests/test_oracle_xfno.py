"""Pins of the oracle's XFNO (oracle/xfno.py) against closed forms and the
invariances of the FNO construction (Section 1.2).

The extrapolated values themselves are parity unpinned (the paper's formula
is in its unavailable supplement); what is fixed here is the fit (exactly
linear data, two points, constant data, order of the points) and each
threshold's energies at OCCT = 1, where no orbital is dropped and the FNO
transformation is a rotation of the virtuals that leaves CCSDT, EOM and MP2
energies unchanged.
"""
import numpy as np
import pytest

from oracle import cc, fno, xfno
from synthetic import make_hamiltonian

PAPER_OCCT = (0.995, 0.9975, 0.999)  # thresholds of the paper's M3 values


def test_fit_reproduces_exact_lines():
    rng = np.random.default_rng(5)
    for _ in range(20):
        a, b = rng.normal(0, 10, 2)
        y = [a + b * x for x in PAPER_OCCT]
        assert abs(xfno.line_at(PAPER_OCCT, y) - (a + b)) < 1e-9 * (1 + abs(a) + abs(b))


def test_fit_two_points_is_the_line_through_them():
    x0, x1, y0, y1 = 0.995, 0.999, -1.25, -1.2625
    ref = y0 + (y1 - y0) * (1.0 - x0) / (x1 - x0)
    assert abs(xfno.line_at([x0, x1], [y0, y1]) - ref) < 1e-13


def test_fit_constant_and_order():
    assert abs(xfno.line_at(PAPER_OCCT, [-3.5] * 3) + 3.5) < 1e-14
    y = [-1.0, -1.1, -1.15]
    assert abs(xfno.line_at(PAPER_OCCT, y) - xfno.line_at(PAPER_OCCT[::-1], y[::-1])) < 1e-13
    with pytest.raises(ValueError):
        xfno.line_at([0.99], [1.0])


def test_full_threshold_reproduces_the_untruncated_energies():
    """OCCT = 1 keeps every virtual: the ground-state, IP target and MP2
    energies equal those of the untransformed problem."""
    h = make_hamiltonian(3, 7, 11, decay=3.0)
    r = xfno.xfno(h.fock, h.eri, 3, [1.0, 0.999], kind="IP", nroots=2)
    p = r["points"][0]
    assert p["kept"] == 7
    full = cc.solve_ccsdt(h.fock, h.eri, 3)
    assert abs(p["e_cc"] - full["e_tot"]) < 1e-9
    w, _, _ = cc.eom_roots_dense(h.fock, h.eri, 3, full["amps"], "IP", 2)
    assert np.max(np.abs(p["e_eom"] - (full["e_tot"] + np.real(w)))) < 1e-8
    assert abs(p["e_mp2_trunc"] - fno.mp2_energy(h.fock, h.eri, 3)) < 1e-12


def test_decay_option_keeps_the_integral_symmetries():
    h = make_hamiltonian(3, 6, 4, decay=2.0)
    g = h.eri
    assert np.allclose(g, -g.transpose(1, 0, 2, 3), atol=1e-15)
    assert np.allclose(g, -g.transpose(0, 1, 3, 2), atol=1e-15)
    assert np.allclose(g, g.transpose(2, 3, 0, 1), atol=1e-15)
    occ, _ = fno.natural_orbitals(h.fock, h.eri, 3)
    assert occ[0] > 10 * occ[-1]
