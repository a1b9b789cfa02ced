"""GPU parity of the left-hand EOM-CCSDT sigma (fno_eom_sigma_left) and of the
left eigenvectors (fno_eom_vectors, left = 1) against the CPU oracle.

The left sigma is the transpose, in the packed basis, of the right sigma;
the GPU runs the transposed term program (reverse order, adjoint tensors,
coefficients corrected for the engine's antisymmetrizer convention).
Tolerances: left-sigma elements to 1e-11 relative to the largest element
(as the right sigma); the adjoint identity <l, sigma(r)> = <sigma_left(l), r>
to 1e-11 relative; left roots equal to the right roots and to the oracle's
dense roots within 1e-8 Eh; left vectors parallel to the oracle's dense left
eigenvectors (|cos| within 1e-7 of 1) and biorthogonal to the GPU's right
vectors of the other roots (|l_i . r_j| < 1e-6 |l_i . r_i|).
"""
import numpy as np
import pytest

from synthetic import make_hamiltonian
from oracle import cc, wick
from tests.helpers import random_amps, random_antisym
from tests.packing import pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2509_14157_amd as P
    return P


def _ctx(P, h, o):
    c = P.Context(0)
    c.load_hamiltonian(h.fock, h.eri, o)
    return c


def _set(c, amps):
    c.set_amplitudes(1, amps[1].ravel())
    c.set_amplitudes(2, pack(amps[2], 2, 2))
    c.set_amplitudes(3, pack(amps[3], 3, 3))


@pytest.mark.parametrize("kind,o,v,seed", [("IP", 3, 5, 1), ("EA", 3, 5, 2), ("IP", 4, 6, 3), ("EA", 2, 7, 4),
                                           ("DIP", 4, 5, 7), ("DEA", 2, 6, 9)])
def test_left_sigma_matches_oracle(P, kind, o, v, seed):
    print(f"left sigma parity {kind} o={o} v={v}", flush=True)
    h = make_hamiltonian(o, v, seed)
    rng = np.random.default_rng(seed)
    amps = random_amps(rng, o, v)
    _, blocks = wick.EOM_SPACES[kind]
    lb = {b: random_antisym(rng, o, v, b[0], b[1], 1.0) for b in blocks}
    lvec = np.concatenate([pack(lb[b], *b) for b in blocks])
    with _ctx(P, h, o) as c:
        _set(c, amps)
        sig = c.eom_sigma_left(kind, lvec)
    ref = cc.eom_sigma_left(h.fock, h.eri, o, amps, kind, lb)
    refv = np.concatenate([pack(ref[b], *b) for b in blocks])
    assert np.abs(sig - refv).max() < 1e-11 * max(1.0, np.abs(refv).max())


@pytest.mark.parametrize("kind,o,v,seed", [("IP", 6, 14, 11), ("EA", 5, 14, 12), ("DIP", 6, 9, 13),
                                           ("DEA", 4, 10, 14)])
def test_adjoint_identity(P, kind, o, v, seed):
    """<l, sigma(r)> = <sigma_left(l), r> at sizes beyond the dense oracle,
    FP64 and FP32 (the R3 products of both sides in FP32)."""
    print(f"adjoint identity {kind} o={o} v={v}", flush=True)
    h = make_hamiltonian(o, v, seed)
    rng = np.random.default_rng(seed)
    amps = random_amps(rng, o, v)
    with _ctx(P, h, o) as c:
        _set(c, amps)
        n = c.eom_size(kind)
        lv, rv = rng.normal(size=n), rng.normal(size=n)
        for prec, tol in (("fp64", 1e-11), ("fp32", 1e-5)):
            a = lv @ c.eom_sigma(kind, rv, prec=prec)
            b = c.eom_sigma_left(kind, lv, prec=prec) @ rv
            assert abs(a - b) < tol * max(1.0, abs(a)), (prec, a, b)


@pytest.mark.parametrize("kind,o,v,seed", [("IP", 4, 6, 21), ("EA", 3, 6, 22), ("DIP", 4, 5, 23), ("DEA", 2, 6, 24)])
def test_left_vectors_match_oracle(P, kind, o, v, seed):
    print(f"left vectors {kind} o={o} v={v}", flush=True)
    h = make_hamiltonian(o, v, seed)
    nroots = 3
    with _ctx(P, h, o) as c:
        c.ccsdt(r_tol=1e-11, e_tol=1e-13)
        amps = {1: c.get_amplitudes(1).reshape(o, v)}
        right = c.eom_vectors(kind, nroots=nroots, r_tol=1e-9, e_tol=1e-11)
        left = c.eom_vectors(kind, nroots=nroots, left=True, r_tol=1e-9, e_tol=1e-11)
        t2, t3 = c.get_amplitudes(2), c.get_amplitudes(3)
    assert right["converged"] and left["converged"]
    assert np.abs(left["omega"] - right["omega"]).max() < 1e-8
    from tests.packing import unpack_fast
    amps[2] = unpack_fast(t2, o, v, 2, 2)
    amps[3] = unpack_fast(t3, o, v, 3, 3)
    w, L, M, sp = cc.eom_left_dense(h.fock, h.eri, o, amps, kind, nroots)
    assert np.abs(left["omega"] - w.real).max() < 1e-8
    _, blocks = wick.EOM_SPACES[kind]
    for k in range(nroots):
        lref = np.concatenate([pack(L[k][b], *b) for b in blocks])
        lref /= np.linalg.norm(lref)
        assert abs(abs(left["vectors"][k] @ lref) - 1.0) < 1e-7
    # biorthogonality of left and right vectors of different roots
    S = left["vectors"] @ right["vectors"].T
    for i in range(nroots):
        for j in range(nroots):
            if i != j:
                assert abs(S[i, j]) < 1e-6 * abs(S[i, i])
