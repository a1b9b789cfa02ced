"""Pins of the learned-guess oracle (oracle/mlp.py) on the CPU.

* backpropagation equals central finite differences of the loss;
* the T1-dressed one-body diagonal equals determinant-space expectation
  values of e^{-T1} H e^{T1} (one hole: E0 - f^_ii; one particle: E0 + f^_aa);
* with T2 (and T3) as well, the full diagonal fo / fv equals the diagonal of
  the one-hole / one-particle block of e^{-T} H e^{T} - E_CC in the N-1 / N+1
  determinant sectors (the 1h-1h block of the EOM-IP matrix and the 1p-1p
  block of the EOM-EA matrix; T3 cannot reach these blocks);
* the MP-style guess has MP2 doubles (a closed form).
"""
import numpy as np

from oracle import det, fno, mlp
from synthetic import make_hamiltonian
from tests.helpers import random_antisym


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.2, mlp.F * mlp.H + mlp.H + mlp.H * mlp.H + mlp.H + mlp.H * mlp.O + mlp.O)
    X = rng.normal(0, 1, (6, mlp.F))
    T = rng.normal(0, 1, (6, mlp.O))
    w = (1.0, 0.5)
    loss, g = mlp.loss_grad(p, X, T, w)
    assert abs(loss - mlp.loss_only(p, X, T, w)) < 1e-14
    idx = rng.choice(p.size, 300, replace=False)
    h = 1e-5
    for i in idx:
        q = p.copy()
        q[i] += h
        lp = mlp.loss_only(q, X, T, w)
        q[i] -= 2 * h
        lm = mlp.loss_only(q, X, T, w)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g[i])), i


def test_dressed_one_body_diagonal_matches_determinants():
    o, v = 3, 4
    h = make_hamiltonian(o, v, 12)
    t1 = random_antisym(np.random.default_rng(3), o, v, 1, 1, 0.1)
    f, _ = mlp.dressed_hamiltonian(h.fock, h.eri, o, t1)
    m = det.DetModel(h.fock, h.eri, o)
    amps = {1: t1}
    x0 = m.reference_vector()
    e0 = float(x0 @ m.similarity(o, amps)(x0))
    for i in range(o):
        s = m.sector(o - 1)
        xi = np.zeros(s.dim)
        xi[s.det_of([k for k in range(o) if k != i])] = 1.0
        assert abs((e0 - float(xi @ m.similarity(o - 1, amps)(xi))) - f[i, i]) < 1e-12
    for a in range(v):
        s = m.sector(o + 1)
        xa = np.zeros(s.dim)
        xa[s.det_of(list(range(o)) + [o + a])] = 1.0
        assert abs((float(xa @ m.similarity(o + 1, amps)(xa)) - e0) - f[o + a, o + a]) < 1e-12


def test_mp_guess_triples_are_determinant_residual_over_denominator():
    """T3 of the guess = <ijk abc| e^{-T} H e^{T} |0> at T = (0, MP2, 0), over D3,
    with the residual taken from the determinant model (independent of Wick)."""
    o, v = 3, 4
    h = make_hamiltonian(o, v, 13)
    g = mlp.mp_guess(h.fock, h.eri, o)
    t2 = fno.mp2_amplitudes(h.fock, h.eri, o)
    m = det.DetModel(h.fock, h.eri, o)
    ref, _ = m.cc_residual({2: t2}, ranks=(3,))
    labels, vals = ref[3]
    eo, ev = np.diag(h.fock)[:o], np.diag(h.fock)[o:]
    for (holes, parts), r in zip(labels, vals):
        d = eo[list(holes)].sum() - ev[[p - o for p in parts]].sum()
        assert abs(g[3][tuple(holes) + tuple(p - o for p in parts)] - r / d) < 1e-13


def test_dressed_diagonal_with_doubles_matches_determinants():
    """fo_i = E0 - <Phi_i| e^{-T} H e^{T} |Phi_i> and fv_a = <Phi^a| e^{-T} H e^{T} |Phi^a> - E0
    for random T1, T2 (and T3, which must not change them), E0 = <0| e^{-T} H e^{T} |0>,
    all in the determinant model (N-1 and N+1 electron sectors)."""
    o, v = 3, 4
    h = make_hamiltonian(o, v, 14)
    rng = np.random.default_rng(5)
    t1 = random_antisym(rng, o, v, 1, 1, 0.1)
    t2 = random_antisym(rng, o, v, 2, 2, 0.08)
    t3 = random_antisym(rng, o, v, 3, 3, 0.05)
    fo, fv = mlp.dressed_diagonal(h.fock, h.eri, o, {1: t1, 2: t2})
    # the T2 part is not small here: a dropped term or a wrong sign shows
    fo1, fv1 = mlp.dressed_diagonal(h.fock, h.eri, o, {1: t1, 2: 0 * t2})
    assert np.abs(fo - fo1).max() > 1e-3 and np.abs(fv - fv1).max() > 1e-3
    m = det.DetModel(h.fock, h.eri, o)
    for amps in ({1: t1, 2: t2}, {1: t1, 2: t2, 3: t3}):
        x0 = m.reference_vector()
        e0 = float(x0 @ m.similarity(o, amps)(x0))
        for i in range(o):
            s = m.sector(o - 1)
            xi = np.zeros(s.dim)
            xi[s.det_of([k for k in range(o) if k != i])] = 1.0
            assert abs((e0 - float(xi @ m.similarity(o - 1, amps)(xi))) - fo[i]) < 1e-12, i
        for a in range(v):
            s = m.sector(o + 1)
            xa = np.zeros(s.dim)
            xa[s.det_of(list(range(o)) + [o + a])] = 1.0
            assert abs((float(xa @ m.similarity(o + 1, amps)(xa)) - e0) - fv[a]) < 1e-12, a
