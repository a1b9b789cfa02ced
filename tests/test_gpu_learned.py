"""Learned guess on the GPU against the FP64 oracle: FP32 gradients of the
network, its BF16 inference, the collected features and targets, and the
learned start of the CCSDT iterations (same energy; plain fallback)."""
import numpy as np
import pytest

from oracle import cc, mlp
from synthetic import make_hamiltonian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2509_14157_amd as P
    return P


def test_gradient_matches_oracle(P):
    print("mlp gradient", flush=True)
    rng = np.random.default_rng(1)
    X = rng.normal(0, 1, (64, 9)).astype(np.float32)
    T = rng.normal(0, 0.3, (64, 2)).astype(np.float32)
    with P.Mlp(0) as net:
        p = rng.normal(0, 0.08, net.num_params).astype(np.float32)
        net.set_params(p)
        loss, g = net.loss_grad(X, T)
    lref, gref = mlp.loss_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lref) < 1e-4 * max(1.0, abs(lref))
    assert np.linalg.norm(g - gref) < 1e-4 * np.linalg.norm(gref)


def test_bf16_inference_matches_oracle(P):
    print("mlp bf16 inference", flush=True)
    rng = np.random.default_rng(2)
    X = rng.normal(0, 1, (3000, 9)).astype(np.float32)
    with P.Mlp(0) as net:
        p = rng.normal(0, 0.08, net.num_params).astype(np.float32)
        net.set_params(p)
        Y = net.predict(X)
    Yr = mlp.forward(p.astype(np.float64), X.astype(np.float64))
    # single-BF16 operands (8 significant bits) through three layers
    assert np.abs(Y - Yr).max() < 0.03 * np.abs(Yr).max() + 1e-3


def test_collected_samples_match_oracle(P):
    print("mlp samples", flush=True)
    o, v = 4, 8
    h = make_hamiltonian(o, v, 51)
    ref = cc.solve_ccsdt(h.fock, h.eri, o, r_tol=1e-11, e_tol=1e-13)
    x3 = mlp.mp_guess(h.fock, h.eri, o)[3]
    fo, fv = mlp.dressed_diagonal(h.fock, h.eri, o, ref["amps"])
    Xr, Tr, _ = mlp.samples(h.fock, h.eri, o, x3, ref["amps"][3], fo, fv)
    with P.Context(0) as c, P.Mlp(0) as net:
        c.load_hamiltonian(h.fock, h.eri, o)
        c.ccsdt(r_tol=1e-11, e_tol=1e-13)
        net.collect(c, 10 ** 9)
        X, T = net.dataset()
    assert X.shape == Xr.shape
    assert np.abs(X - Xr).max() < 1e-5 * max(1.0, np.abs(Xr).max())
    assert np.abs(T - Tr).max() < 1e-5 * max(1.0, np.abs(Tr).max())


def test_learned_start_reaches_the_same_energy(P):
    print("learned start", flush=True)
    with P.Mlp(0) as net:
        for seed in (60, 61, 62, 63):
            h = make_hamiltonian(4, 12, seed)
            with P.Context(0) as c:
                c.load_hamiltonian(h.fock, h.eri, 4)
                c.ccsdt(r_tol=1e-10, e_tol=1e-12)
                net.collect(c, 1 << 14)
        loss = net.train(400, batch=1024, lr=1e-3, seed=7)
        assert np.isfinite(loss)
        h = make_hamiltonian(4, 12, 70)
        with P.Context(0) as c:
            c.load_hamiltonian(h.fock, h.eri, 4)
            plain = c.ccsdt(r_tol=1e-9, e_tol=1e-11)
            c.set_guess_model(net)
            learned = c.ccsdt(r_tol=1e-9, e_tol=1e-11, guess=1)
            accepted = c.last_guess_accepted()
    print(f"iterations plain {plain['iters']} learned {learned['iters']} (accepted: {accepted}), loss {loss:.3e}")
    assert learned["converged"]
    assert abs(learned["e_tot"] - plain["e_tot"]) < 1e-9
    # a rejected guess costs one residual evaluation at most
    assert learned["iters"] <= plain["iters"] + 1
