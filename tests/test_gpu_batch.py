"""Batched EOM over uneven-size instances, Davidson root blocks, graph replay of
the sigma sweep and the GEMM tile autotuner, against the unbatched paths.

Batched instances compute exactly what the single-instance solver computes (same
kernels in the same order on each context): roots and iteration counts must be
bitwise equal.  Root blocks change GEMM shapes (rounding only): 1e-10 Eh.
"""
import numpy as np
import pytest

from synthetic import make_hamiltonian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2509_14157_amd as P
    return P


def _solved(P, o, v, seed):
    h = make_hamiltonian(o, v, seed)
    c = P.Context(0)
    c.load_hamiltonian(h.fock, h.eri, o)
    c.ccsdt(r_tol=1e-9, e_tol=1e-11)
    return c


@pytest.mark.parametrize("kind", ["IP", "EA", "DIP", "DEA"])
def test_batch_matches_single(P, kind):
    print(f"batched {kind}", flush=True)
    ctxs = [_solved(P, o, v, s) for o, v, s in [(4, 8, 41), (5, 6, 42), (4, 9, 43)]]
    try:
        single = [c.eom(kind, nroots=3, r_tol=1e-7, e_tol=1e-10) for c in ctxs]
        batch = P.batch_eom(ctxs, kind, nroots=3, r_tol=1e-7, e_tol=1e-10)
        for s, b in zip(single, batch):
            assert s["converged"] and b["converged"]
            assert b["iters"] == s["iters"]
            assert np.array_equal(b["omega"], s["omega"])
    finally:
        for c in ctxs:
            c.close()


@pytest.mark.parametrize("kind", ["EA", "DIP"])
def test_root_block_matches_single_vectors(P, kind):
    print(f"root block {kind}", flush=True)
    c = _solved(P, 5, 8, 44)
    with c:
        one = c.eom(kind, nroots=4, r_tol=1e-8, e_tol=1e-11, block=1)
        blk = c.eom(kind, nroots=4, r_tol=1e-8, e_tol=1e-11, block=4)
    assert one["converged"] and blk["converged"]
    assert np.abs(np.sort(one["omega"]) - np.sort(blk["omega"])).max() < 1e-10


@pytest.mark.parametrize("kind,prec", [("IP", "fp64"), ("DEA", "fp32")])
def test_sigma_graph_replay_matches_host_launches(P, kind, prec):
    print(f"sigma graph replay {kind} {prec}", flush=True)
    c = _solved(P, 4, 7, 45)
    with c:
        c.set_graphs(False)
        ref = c.eom(kind, nroots=3, r_tol=1e-7, e_tol=1e-10, prec=prec, allow_noconv=True)
        c.set_graphs(True)
        got = c.eom(kind, nroots=3, r_tol=1e-7, e_tol=1e-10, prec=prec, allow_noconv=True)
    assert got["iters"] == ref["iters"]
    assert np.array_equal(got["omega"], ref["omega"])


def test_autotuned_tiles_give_the_same_energy(P):
    print("autotune", flush=True)
    h = make_hamiltonian(6, 20, 46)
    with P.Context(0) as c:
        c.load_hamiltonian(h.fock, h.eri, 6)
        e0 = c.ccsdt(r_tol=1e-9, e_tol=1e-11)["e_tot"]
        c.set_autotune(True)
        c.profile(True)
        e1 = c.ccsdt(r_tol=1e-9, e_tol=1e-11)["e_tot"]
        rep = c.profile_report()
        c.profile(False)
    assert abs(e1 - e0) < 1e-10
    assert len(rep["tuned"]) > 0


def test_autotune_setting_survives_truncation(P):
    print("autotune after truncation", flush=True)
    h = make_hamiltonian(4, 12, 47)
    with P.Context(0) as c:
        c.set_autotune(True)  # before the engine is rebuilt by the truncation
        c.load_hamiltonian(h.fock, h.eri, 4)
        kept, _, _ = c.truncate(1.0, 9)
        assert kept == 9
        c.profile(True)
        c.ccsdt(max_iter=1, allow_noconv=True)
        rep = c.profile_report()
        c.profile(False)
    assert len(rep["tuned"]) > 0


@pytest.mark.parametrize("kind,prec", [("IP", "fp64"), ("EA", "fp64"), ("DIP", "fp64"), ("DEA", "fp32")])
def test_grouped_batch_matches_grouped_single(P, kind, prec):
    """fno_batch_eom_grouped: per sigma round and term, the GEMMs of every instance in
    one persistent launch per kernel instantiation, tiles taken from a device work
    queue.  Each instance's roots and iteration count are bitwise those of a grouped
    batch that holds that instance alone (the grouping changes nothing), and agree
    with fno_eom's (which may split K and so rounds differently): 1e-9 Eh in FP64,
    1e-6 Eh with FP32 triples products."""
    print(f"grouped batch {kind} {prec}", flush=True)
    ctxs = [_solved(P, o, v, s) for o, v, s in [(4, 8, 41), (5, 6, 42), (4, 9, 43), (6, 10, 46)]]
    try:
        kw = dict(nroots=3, r_tol=1e-7, e_tol=1e-10, prec=prec)
        alone = [P.batch_eom([c], kind, grouped=True, **kw)[0] for c in ctxs]
        group = P.batch_eom(ctxs, kind, grouped=True, **kw)
        single = [c.eom(kind, **kw) for c in ctxs]
        tol = 1e-9 if prec == "fp64" else 1e-6
        for a, g, s in zip(alone, group, single):
            assert a["converged"] and g["converged"] and s["converged"]
            assert g["iters"] == a["iters"]
            assert np.array_equal(g["omega"], a["omega"])
            assert np.abs(g["omega"] - s["omega"]).max() < tol, (g["omega"], s["omega"])
    finally:
        for c in ctxs:
            c.close()
