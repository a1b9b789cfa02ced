"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: they compare the Wick-expanded
algebra with the determinant-space definitions (eqs 1-7), with exact FCI
where the method is exact, with closed forms of eqs 8-10, and with
invariances the FNO construction (Section 1.2) guarantees.
"""
import json
import os

import numpy as np
import pytest

from synthetic import make_hamiltonian
from oracle import cc, det, fno, wick
from tests.helpers import random_amps, random_antisym

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ generator
def test_generator_symmetry_and_determinism():
    h = make_hamiltonian(3, 5, 7)
    g = h.eri
    assert np.allclose(g, -g.transpose(1, 0, 2, 3), atol=1e-15)
    assert np.allclose(g, -g.transpose(0, 1, 3, 2), atol=1e-15)
    assert np.allclose(g, g.transpose(2, 3, 0, 1), atol=1e-15)
    assert np.allclose(h.fock, np.diag(np.diag(h.fock)))
    eo, ev = np.diag(h.fock)[:3], np.diag(h.fock)[3:]
    assert np.all(np.diff(eo) >= 0) and np.all(np.diff(ev) >= 0)
    assert eo.max() <= -0.5 and eo.min() >= -2.0 and ev.min() >= 0.3 and ev.max() <= 3.0
    assert make_hamiltonian(3, 5, 7).sha256() == h.sha256()


def test_generator_golden_hashes():
    with open(os.path.join(GOLDEN, "synthetic_sha256.json")) as f:
        ref = json.load(f)
    for key, digest in ref.items():
        o, v, seed, lo, hi = key.split(",")
        h = make_hamiltonian(int(o), int(v), int(seed), evir=(float(lo), float(hi)))
        assert h.sha256() == digest, key


# ------------------------------------------------------------ determinant model
def test_reference_energy_is_expectation_value():
    h = make_hamiltonian(3, 4, 3)
    m = det.DetModel(h.fock, h.eri, 3)
    x = m.reference_vector()
    assert abs(x @ (m.H(3) @ x) - cc.reference_energy(h.fock, h.eri, 3)) < 1e-13
    Hd = m.H(3).toarray()
    assert np.allclose(Hd, Hd.T, atol=1e-14)
    # variational bound
    assert m.fci(3)[0] <= cc.reference_energy(h.fock, h.eri, 3) + 1e-14


def test_fock_is_fock_of_reference():
    # <Phi_i^a|H|Phi_0> = f_ai (Brillouin): zero for the diagonal synthetic Fock matrix
    h = make_hamiltonian(3, 4, 8)
    h.fock[0, 4] = h.fock[4, 0] = 0.03
    m = det.DetModel(h.fock, h.eri, 3)
    res, _ = m.cc_residual({1: np.zeros((3, 4)), 2: np.zeros((3, 3, 4, 4))}, ranks=(1,))
    labels, vals = res[1]
    for (holes, parts), val in zip(labels, vals):
        assert abs(val - h.fock[parts[0], holes[0]]) < 1e-14


# ------------------------------------------------------------ Wick algebra vs definitions
@pytest.mark.parametrize("o,v,seed", [(3, 5, 7), (4, 4, 9)])
def test_cc_residual_matches_determinant_definition(o, v, seed):
    h = make_hamiltonian(o, v, seed)
    rng = np.random.default_rng(seed)
    amps = random_amps(rng, o, v)
    m = det.DetModel(h.fock, h.eri, o)
    ref, e_det = m.cc_residual(amps)
    R = cc.cc_residual(h.fock, h.eri, o, amps)
    for k in (1, 2, 3):
        labels, vals = ref[k]
        got = det.unique_from_dense(R[k], labels, o)
        assert np.abs(got - vals).max() < 1e-12 * max(1.0, np.abs(vals).max())
    e = cc.cc_energy(h.fock, h.eri, o, amps) + cc.reference_energy(h.fock, h.eri, o)
    assert abs(e - e_det) < 1e-12


def test_cc_residual_element_matches_dense():
    h = make_hamiltonian(3, 5, 4)
    amps = random_amps(np.random.default_rng(4), 3, 5)
    R = cc.cc_residual(h.fock, h.eri, 3, amps)
    for idx in [(0, 1, 2, 0, 2, 4), (0, 1, 2, 1, 3, 4), (0, 2, 1, 4, 0, 3)]:
        assert abs(cc.cc_residual_element(h.fock, h.eri, 3, amps, 3, idx) - R[3][idx]) < 1e-12


@pytest.mark.parametrize("kind,o,v", [("IP", 3, 4), ("EA", 3, 4), ("DIP", 4, 3), ("DEA", 2, 5)])
def test_eom_sigma_matches_commutator_definition(kind, o, v):
    h = make_hamiltonian(o, v, 11)
    rng = np.random.default_rng(1)
    amps = random_amps(rng, o, v)
    _, blocks = wick.EOM_SPACES[kind]
    rb = {b: random_antisym(rng, o, v, b[0], b[1], 1.0) for b in blocks}
    m = det.DetModel(h.fock, h.eri, o)
    ref = m.eom_sigma(kind, amps, rb)
    got = cc.eom_sigma(h.fock, h.eri, o, amps, kind, rb)
    for blk, labels, vals in ref:
        if not labels:
            continue
        g = det.unique_from_dense(got[blk], labels, o)
        assert np.abs(g - vals).max() < 1e-11 * max(1.0, np.abs(vals).max()), blk


# ------------------------------------------------------------ exactness (FCI)
def test_ccsdt_exact_for_three_electrons():
    h = make_hamiltonian(3, 5, 21)
    r = cc.solve_ccsdt(h.fock, h.eri, 3, r_tol=1e-11, e_tol=1e-13)
    assert r["converged"]
    assert abs(r["e_tot"] - det.DetModel(h.fock, h.eri, 3).fci(3)[0]) < 1e-10


@pytest.fixture(scope="module")
def n4_problem():
    h = make_hamiltonian(4, 4, 23)
    r = cc.solve_ccsdt(h.fock, h.eri, 4, r_tol=1e-11, e_tol=1e-13)
    return h, r, det.DetModel(h.fock, h.eri, 4)


def test_dip_exact_for_four_electrons(n4_problem):
    # the 2h/3h1p/4h2p space spans every 2-electron determinant of a 4-electron reference
    h, r, m = n4_problem
    w, _, _ = cc.eom_roots_dense(h.fock, h.eri, 4, r["amps"], "DIP", 6)
    assert np.abs(w.imag).max() < 1e-10
    assert np.abs(w.real + r["e_tot"] - m.fci(2)[:6]).max() < 1e-9


def test_ip_not_exact_for_four_electrons(n4_problem):
    # 4h3p is missing from IP-EOM-CCSDT, so a 4-electron reference must show a deviation
    h, r, m = n4_problem
    w, _, _ = cc.eom_roots_dense(h.fock, h.eri, 4, r["amps"], "IP", 4)
    dev = np.abs(w.real + r["e_tot"] - m.fci(3)[:4]).max()
    assert 1e-9 < dev < 1e-3


def test_ip_exact_for_three_electrons():
    h = make_hamiltonian(3, 5, 21)
    r = cc.solve_ccsdt(h.fock, h.eri, 3, r_tol=1e-11, e_tol=1e-13)
    w, _, _ = cc.eom_roots_dense(h.fock, h.eri, 3, r["amps"], "IP", 5)
    assert np.abs(w.real + r["e_tot"] - det.DetModel(h.fock, h.eri, 3).fci(2)[:5]).max() < 1e-9


@pytest.mark.parametrize("kind,nel", [("EA", 3), ("DEA", 4)])
def test_ea_dea_exact_for_two_electrons(kind, nel):
    h = make_hamiltonian(2, 6, 22)
    r = cc.solve_ccsdt(h.fock, h.eri, 2, r_tol=1e-11, e_tol=1e-13)
    w, _, _ = cc.eom_roots_dense(h.fock, h.eri, 2, r["amps"], kind, 4)
    assert np.abs(w.real + r["e_tot"] - det.DetModel(h.fock, h.eri, 2).fci(nel)[:4]).max() < 1e-9


def test_ccsdt_error_is_fifth_order():
    # CCSDT is exact through fourth order in the fluctuation potential: scaling
    # <pq||rs> by lam with the Fock operator fixed gives E_CCSDT - E_FCI = O(lam^5)
    h = make_hamiltonian(4, 6, 31, sigma=0.25)
    errs = []
    lams = (0.3, 0.6)
    for lam in lams:
        eri = lam * h.eri
        r = cc.solve_ccsdt(h.fock, eri, 4, r_tol=1e-12, e_tol=1e-14, max_iter=200)
        assert r["converged"]
        e_fci = det.DetModel(h.fock, eri, 4).fci(4)[0]
        errs.append(abs(r["e_tot"] - e_fci))
    slope = np.log(errs[1] / errs[0]) / np.log(lams[1] / lams[0])
    assert 4.4 < slope < 6.0, (errs, slope)


# ------------------------------------------------------------ MP2 / FNO (eqs 8-10)
def test_first_jacobi_step_is_mp2():
    h = make_hamiltonian(4, 8, 5)
    r = cc.solve_ccsdt(h.fock, h.eri, 4, max_iter=1, diis_n=0)
    t2 = fno.mp2_amplitudes(h.fock, h.eri, 4)
    assert np.abs(r["amps"][2] - t2).max() < 1e-14
    assert np.abs(r["amps"][1]).max() < 1e-15 and np.abs(r["amps"][3]).max() < 1e-15
    assert abs(r["e_corr"] - fno.mp2_energy(h.fock, h.eri, 4)) < 1e-13


def test_virtual_density_properties():
    h = make_hamiltonian(4, 10, 6)
    D = fno.virtual_density(h.fock, h.eri, 4)
    t = fno.mp2_amplitudes(h.fock, h.eri, 4)
    assert np.allclose(D, D.T, atol=1e-15)
    assert np.linalg.eigvalsh(D).min() > -1e-15
    assert abs(np.trace(D) - 0.5 * np.sum(t * t)) < 1e-14
    # brute-force element by element from eq (10)
    o, v = 4, 10
    g = h.eri
    e = np.diag(h.fock)
    a, b = 2, 7
    s = 0.0
    for c in range(v):
        for i in range(o):
            for j in range(o):
                if i == j:
                    continue
                num = g[o + c, o + b, i, j] * g[i, j, o + c, o + a]
                s += num / ((e[i] + e[j] - e[o + c] - e[o + b]) * (e[i] + e[j] - e[o + c] - e[o + a]))
    assert abs(0.5 * s - D[a, b]) < 1e-15


def test_occt_cut_rules():
    occ = np.array([0.4, 0.3, 0.2, 0.1])
    assert fno.occt_cut(occ, 1.0) == 4
    assert fno.occt_cut(occ, 0.7) == 2
    assert fno.occt_cut(occ, 0.70000001) == 3
    assert fno.occt_cut(occ, 0.4) == 1
    # a degenerate pair straddling the cut is kept whole
    assert fno.occt_cut(np.array([0.4, 0.25, 0.25, 0.1]), 0.6) == 3
    with pytest.raises(ValueError):
        fno.occt_cut(occ, 0.0)
    h = make_hamiltonian(4, 14, 2, evir=(0.2, 6.0))
    occ, _ = fno.natural_orbitals(h.fock, h.eri, 4)
    ks = [fno.occt_cut(occ, x) for x in (0.5, 0.8, 0.9, 0.95, 0.99, 1.0)]
    assert ks == sorted(ks) and ks[-1] == 14
    assert np.all(np.diff(occ) <= 0)


def test_fno_full_space_reproduces_canonical():
    h = make_hamiltonian(3, 6, 12)
    r0 = cc.solve_ccsdt(h.fock, h.eri, 3, r_tol=1e-11, e_tol=1e-13)
    tr = fno.truncate(h.fock, h.eri, 3, occt=1.0)
    assert tr["nvir"] == 6
    fv = tr["fock"][3:, 3:]
    assert np.allclose(fv, np.diag(np.diag(fv)), atol=1e-13)
    assert np.all(np.diff(np.diag(fv)) >= -1e-14)
    r1 = cc.solve_ccsdt(tr["fock"], tr["eri"], 3, r_tol=1e-11, e_tol=1e-13)
    assert abs(r0["e_tot"] - r1["e_tot"]) < 1e-10
    w0, _, _ = cc.eom_roots_dense(h.fock, h.eri, 3, r0["amps"], "EA", 3)
    w1, _, _ = cc.eom_roots_dense(tr["fock"], tr["eri"], 3, r1["amps"], "EA", 3)
    assert np.abs(w0.real - w1.real).max() < 1e-9


def test_fno_invariant_to_virtual_rotation():
    # NOs are defined by the density, not by the canonical virtual basis: a
    # random orthogonal rotation of the input virtuals must not change the
    # truncated-space energy (the rotated Fock block is no longer diagonal,
    # so the MP2 step is done in the canonical basis of that block).
    h = make_hamiltonian(3, 7, 13)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(7, 7)))
    tr0 = fno.truncate(h.fock, h.eri, 3, nvir_keep=5)
    full = np.eye(10)
    full[3:, 3:] = Q
    f2 = full.T @ h.fock @ full
    g = h.eri
    for _ in range(4):
        g = np.tensordot(g, full, axes=([0], [0]))
    ev, V = np.linalg.eigh(f2[3:, 3:])
    full2 = np.eye(10)
    full2[3:, 3:] = V
    f3 = full2.T @ f2 @ full2
    for _ in range(4):
        g = np.tensordot(g, full2, axes=([0], [0]))
    tr1 = fno.truncate(f3, g, 3, nvir_keep=5)
    e0 = cc.solve_ccsdt(tr0["fock"], tr0["eri"], 3, r_tol=1e-11, e_tol=1e-13)["e_tot"]
    e1 = cc.solve_ccsdt(tr1["fock"], tr1["eri"], 3, r_tol=1e-11, e_tol=1e-13)["e_tot"]
    assert abs(e0 - e1) < 1e-10


# ------------------------------------------------------------ solvers
def test_davidson_matches_dense_eigenvalues():
    h = make_hamiltonian(4, 5, 17)
    r = cc.solve_ccsdt(h.fock, h.eri, 4, r_tol=1e-10, e_tol=1e-12)
    for kind in ("IP", "EA"):
        w, _, _ = cc.eom_roots_dense(h.fock, h.eri, 4, r["amps"], kind, 3)
        d = cc.davidson(h.fock, h.eri, 4, r["amps"], kind, 3, r_tol=1e-8, e_tol=1e-11)
        assert d["converged"]
        assert np.abs(np.sort(d["omega"]) - w.real).max() < 1e-9


def test_diis_and_plain_jacobi_reach_same_solution():
    h = make_hamiltonian(4, 6, 19)
    a = cc.solve_ccsdt(h.fock, h.eri, 4, r_tol=1e-10, e_tol=1e-12)
    b = cc.solve_ccsdt(h.fock, h.eri, 4, r_tol=1e-10, e_tol=1e-12, diis_n=0, max_iter=300)
    assert a["converged"] and b["converged"]
    assert abs(a["e_tot"] - b["e_tot"]) < 1e-10
    assert a["iters"] <= b["iters"]


# ------------------------------------------------------------ left EOM sigma
@pytest.mark.parametrize("kind,o,v,seed", [("IP", 3, 4, 31), ("EA", 2, 5, 32), ("DIP", 4, 3, 33), ("DEA", 2, 4, 34)])
def test_left_sigma_is_the_transpose(kind, o, v, seed):
    """<l, sigma(r)> = <sigma_left(l), r> over unique elements for random l, r:
    the left sigma is the transpose of the right one (the oracle's right sigma
    is pinned to the determinant commutator above)."""
    h = make_hamiltonian(o, v, seed)
    rng = np.random.default_rng(seed)
    amps = random_amps(rng, o, v)
    _, blocks = wick.EOM_SPACES[kind]
    sp = cc._Space(o, v, list(blocks))
    lv, rv = rng.normal(size=sp.dim), rng.normal(size=sp.dim)
    sig = sp.pack(cc.eom_sigma(h.fock, h.eri, o, amps, kind, sp.unpack(rv)))
    sigl = sp.pack(cc.eom_sigma_left(h.fock, h.eri, o, amps, kind, sp.unpack(lv)))
    assert abs(lv @ sig - sigl @ rv) < 1e-12 * max(1.0, abs(lv @ sig))


def test_left_roots_are_the_fci_energies_for_three_electrons():
    """EOM-IP is exact for three electrons (above): its left eigenvalues, like
    the right ones, are the FCI energies of the two-electron sector."""
    h = make_hamiltonian(3, 5, 21)
    res = cc.solve_ccsdt(h.fock, h.eri, 3, r_tol=1e-12, e_tol=1e-14)
    w, L, M, sp = cc.eom_left_dense(h.fock, h.eri, 3, res["amps"], "IP", 4)
    fci = det.DetModel(h.fock, h.eri, 3).fci(2)[:4]
    assert np.abs(np.sort(res["e_tot"] + w.real) - fci).max() < 1e-9
    for wk, lk in zip(w, L):
        lp = sp.pack(lk)
        assert np.linalg.norm(M.T @ lp - wk.real * lp) < 1e-9
