"""The C ABI's device-pointer calls on a caller's stream, and its error
statuses under bad input (failure injection from the host: every kernel that
runs still exits normally).

* fno_set_amplitudes_dev / fno_cc_residual_dev / fno_eom_sigma_dev on
  caller-allocated device buffers, with the context on a caller-created
  stream (fno_set_stream), give exactly what the host-pointer calls give;
* NaN / Inf in the inputs -> FNO_ENONFINITE; integrals without the
  <pq||rs> symmetry, a non-symmetric Fock matrix, OCCT outside (0, 1] ->
  FNO_EINVAL; calls out of order -> FNO_ESTATE; max_iter = 1 ->
  FNO_ENOCONV with results written; an EOM subspace larger than the device
  -> FNO_ENOMEM (checked before anything is allocated).
"""
import math

import numpy as np
import pytest

from synthetic import make_hamiltonian
from tests.helpers import HipBuffers, random_amps, random_antisym
from tests.packing import pack
from oracle import wick

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2509_14157_amd as P
    return P


def _ctx(P, h):
    c = P.Context(0)
    c.load_hamiltonian(h.fock, h.eri, h.nocc)
    return c


def test_dev_calls_on_a_caller_stream(P):
    print("dev calls on a caller stream", flush=True)
    o, v = 4, 12
    h = make_hamiltonian(o, v, 1)
    rng = np.random.default_rng(4)
    amps = random_amps(rng, o, v)
    packed = [amps[1].ravel(), pack(amps[2], 2, 2), pack(amps[3], 3, 3)]
    _, blocks = wick.EOM_SPACES["EA"]
    rvec = np.concatenate([pack(random_antisym(rng, o, v, b[0], b[1], 1.0), *b) for b in blocks])
    with _ctx(P, h) as c:
        for k in (1, 2, 3):
            c.set_amplitudes(k, packed[k - 1])
        ref = c.cc_residual("fp64")
        sig_ref = c.eom_sigma("EA", rvec)
    hip = HipBuffers()
    with _ctx(P, h) as c:
        s = hip.stream()
        c.set_stream(s)
        t = [hip.upload(x) for x in packed]
        r = [hip.alloc(x.size) for x in packed]
        back = hip.alloc(packed[2].size)
        rt = hip.upload(rvec)
        st = hip.alloc(rvec.size)
        for k in (1, 2, 3):
            c.set_amplitudes_dev(k, t[k - 1], packed[k - 1].size)
        c.get_amplitudes_dev(3, back, packed[2].size)
        ec = c.cc_residual_dev("fp64", r[0], r[1], r[2])
        c.eom_sigma_dev("EA", rt, st, rvec.size)
        hip.sync(s)
        c.set_stream(0)
        got = [hip.download(p, x.size) for p, x in zip(r, packed)]
        got_back = hip.download(back, packed[2].size)
        got_sig = hip.download(st, rvec.size)
    hip.close(s)
    assert np.array_equal(got_back, packed[2])
    for g, e in zip(got, ref[:3]):
        assert np.array_equal(g, e)
    assert ec == ref[3]
    assert np.array_equal(got_sig, sig_ref)


def test_nonfinite_inputs_are_rejected(P):
    h = make_hamiltonian(3, 5, 2)
    with P.Context(0) as c:
        f = h.fock.copy()
        f[1, 1] = np.nan
        with pytest.raises(P.FnoError) as e:
            c.load_hamiltonian(f, h.eri, 3)
        assert e.value.code == P.FNO_ENONFINITE
        g = h.eri.copy()
        g[0, 1, 3, 4] = np.inf
        with pytest.raises(P.FnoError) as e:
            c.load_hamiltonian(h.fock, g, 3)
        assert e.value.code == P.FNO_ENONFINITE
        c.load_hamiltonian(h.fock, h.eri, 3)
        t = np.zeros(3 * 5)
        t[4] = np.nan
        with pytest.raises(P.FnoError) as e:
            c.set_amplitudes(1, t)
        assert e.value.code == P.FNO_ENONFINITE


def test_bad_symmetry_and_options_are_rejected(P):
    h = make_hamiltonian(3, 5, 2)
    with P.Context(0) as c:
        g = h.eri.copy()
        g[0, 1, 3, 4] += 1e-3  # breaks <pq||rs> = -<qp||rs> = <rs||pq>
        with pytest.raises(P.FnoError) as e:
            c.load_hamiltonian(h.fock, g, 3)
        assert e.value.code == P.FNO_EINVAL
        f = h.fock.copy()
        f[0, 5] += 1e-3  # f not symmetric
        with pytest.raises(P.FnoError) as e:
            c.load_hamiltonian(f, h.eri, 3)
        assert e.value.code == P.FNO_EINVAL
        # out of order: truncation before a Hamiltonian
        with pytest.raises(P.FnoError) as e:
            c.truncate(0.9)
        assert e.value.code == P.FNO_ESTATE
        c.load_hamiltonian(h.fock, h.eri, 3)
        for occt in (0.0, -0.5, 1.5):
            with pytest.raises(P.FnoError) as e:
                c.truncate(occt)
            assert e.value.code == P.FNO_EINVAL
        # EOM before a converged ground state
        with pytest.raises(P.FnoError) as e:
            c.eom("IP", nroots=2)
        assert e.value.code == P.FNO_ESTATE


def test_max_iter_one_reports_noconv_with_results(P):
    h = make_hamiltonian(4, 12, 1)
    with _ctx(P, h) as c:
        with pytest.raises(P.FnoError) as e:
            c.ccsdt(max_iter=1)
        assert e.value.code == P.FNO_ENOCONV
        r = c.ccsdt(max_iter=1, allow_noconv=True)
    assert not r["converged"] and r["iters"] == 1
    assert np.isfinite(r["e_tot"]) and r["res_norm"] > 0


def test_eom_larger_than_the_device_is_enomem(P):
    """DEA with 12 electrons in 64 virtuals: 42 million R elements per vector,
    2 x 512 subspace vectors need about 340 GB, more than the device has."""
    print("eom enomem", flush=True)
    o, v = 12, 64
    h = make_hamiltonian(o, v, 5)
    with _ctx(P, h) as c:
        c.ccsdt(max_iter=1, allow_noconv=True)
        assert c.eom_size("DEA") > 40_000_000
        with pytest.raises(P.FnoError) as e:
            c.eom("DEA", nroots=4, max_sub=512, max_iter=2)
        assert e.value.code == P.FNO_ENOMEM
        assert "GB" in str(e.value)


INTERMEDIATES = ("W3_vvvv", "F3_vv", "W3_ovvo", "W3_vvvo", "W3_ovoo", "W3_oooo", "F3_oo")


def triples_dev_inputs(P, o, v, seed):
    """Amplitudes, the context's dressed intermediates at them and the context's R3 (FP64, FP32, split-BF16)."""
    h = make_hamiltonian(o, v, seed)
    amps = random_amps(np.random.default_rng(seed), o, v)
    with _ctx(P, h) as c:
        c.set_amplitudes(1, amps[1].ravel())
        c.set_amplitudes(2, pack(amps[2], 2, 2))
        c.set_amplitudes(3, pack(amps[3], 3, 3))
        r32 = c.cc_residual("fp32")[2]
        rb3 = c.cc_residual("bf16x3")[2]
        r64 = c.cc_residual("fp64")[2]
        arrays = {k: c.debug_tensor(k) for k in INTERMEDIATES}
        arrays["T3"] = c.get_amplitudes(3)
        arrays["T2"] = c.get_amplitudes(2)
    return arrays, {"fp64": r64, "fp32": r32, "bf16x3": rb3}


@pytest.mark.parametrize("o,v", [(4, 12), (7, 24)])
def test_triples_residual_dev_matches_context(P, o, v):
    """The context-free fused triples entry point on device buffers gives the
    context's triples residual bit for bit (same kernels; R3 starts at zero
    in both, and no other term adds to R3)."""
    print(f"triples residual dev o={o} v={v}", flush=True)
    arrays, ref = triples_dev_inputs(P, o, v, 5)
    hip = HipBuffers()
    ptrs = {k: hip.upload(x) for k, x in arrays.items()}
    n3 = arrays["T3"].size
    for prec in ("fp64", "fp32", "bf16x3"):
        r3 = hip.upload(np.zeros(n3))
        P.triples_residual_dev(0, o, v, prec, ptrs, r3)
        assert np.array_equal(hip.download(r3, n3), ref[prec]), prec
    s = hip.stream()
    with pytest.raises(P.FnoError) as e:
        P.triples_residual_dev(0, o, 65, "fp64", ptrs, r3, s)
    assert e.value.code == P.FNO_EINVAL
    hip.close(s)
