"""Python binding of libfnocc (FNO-EOM-CCSDT on MI355X / gfx950).

Argument marshalling only: every step of the computation runs in the HIP
library.  Importing the package does not need a GPU; creating a Context
does, and raises if the library or a gfx950 device is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY_PATH = os.path.join(_HERE, "libfnocc.so")

FNO_OK, FNO_EINVAL, FNO_ENOMEM, FNO_EDEVICE, FNO_ENOCONV, FNO_ENONFINITE, FNO_ESTATE = 0, -1, -2, -3, -4, -5, -6
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
KIND = {"IP": 1, "DIP": 2, "EA": 3, "DEA": 4}

# exported C symbols (kept in sync with include/fnocc.h)
SYMBOLS = ["fno_create", "fno_destroy", "fno_last_error", "fno_set_stream", "fno_load_hamiltonian",
           "fno_truncate", "fno_mp2_energies", "fno_xfno", "fno_cc_opts_default", "fno_ccsdt", "fno_eom_opts_default", "fno_eom", "fno_sizes",
           "fno_get_amplitudes", "fno_set_amplitudes", "fno_amplitude_size", "fno_cc_residual", "fno_eom_size",
           "fno_eom_sigma", "fno_eom_sigma_left", "fno_eom_vectors", "fno_last_flops", "fno_last_trace", "fno_get_amplitudes_dev",
           "fno_set_amplitudes_dev", "fno_cc_residual_dev", "fno_eom_sigma_dev", "fno_triples_residual_dev", "fno_dev_last_error",
           "fno_triples_residual_dev_noalloc", "fno_profile", "fno_profile_report", "fno_profile_filter",
           "fno_set_graphs", "fno_set_fused", "fno_set_autotune", "fno_batch_eom", "fno_batch_eom_grouped", "fno_mlp_num_params", "fno_mlp_create",
           "fno_mlp_destroy", "fno_mlp_last_error", "fno_mlp_collect", "fno_mlp_samples", "fno_mlp_train",
           "fno_mlp_save", "fno_mlp_load", "fno_mlp_params", "fno_mlp_loss_grad", "fno_mlp_predict", "fno_mlp_dataset",
           "fno_set_guess_model", "fno_last_guess_accepted", "fno_debug_tensor_size", "fno_debug_tensor", "fno_debug_gemm"]


class FnoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class CCOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("r_tol", C.c_double), ("e_tol", C.c_double), ("diis_n", C.c_int),
                ("diis_start", C.c_int), ("prec", C.c_int), ("guess", C.c_int)]


class EOMOpts(C.Structure):
    _fields_ = [("nroots", C.c_int), ("max_iter", C.c_int), ("max_sub", C.c_int), ("e_tol", C.c_double),
                ("r_tol", C.c_double), ("prec", C.c_int), ("guess", C.c_int), ("precond", C.c_int),
                ("block", C.c_int)]


_lib = None


def library() -> C.CDLL:
    """Load libfnocc.so (built in-tree by __graft_entry__.build or paper_2509_14157_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY_PATH):
            raise ImportError(f"{LIBRARY_PATH} is missing: build it with python -m paper_2509_14157_amd.build")
        lib = C.CDLL(LIBRARY_PATH)
        dp = C.POINTER(C.c_double)
        lib.fno_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
        lib.fno_destroy.argtypes = [C.c_void_p]
        lib.fno_destroy.restype = None
        lib.fno_last_error.argtypes = [C.c_void_p]
        lib.fno_last_error.restype = C.c_char_p
        lib.fno_set_stream.argtypes = [C.c_void_p, C.c_void_p]
        lib.fno_load_hamiltonian.argtypes = [C.c_void_p, C.c_int, C.c_int, dp, dp, C.c_double]
        lib.fno_truncate.argtypes = [C.c_void_p, C.c_double, C.c_int, C.POINTER(C.c_int), dp, dp]
        lib.fno_mp2_energies.argtypes = [C.c_void_p, dp, dp]
        lib.fno_xfno.argtypes = [C.c_void_p, C.c_int, dp, C.POINTER(CCOpts), C.c_int, C.POINTER(EOMOpts),
                                 C.POINTER(C.c_int), dp, dp, dp, dp]
        lib.fno_cc_opts_default.argtypes = [C.POINTER(CCOpts)]
        lib.fno_cc_opts_default.restype = None
        lib.fno_ccsdt.argtypes = [C.c_void_p, C.POINTER(CCOpts), dp, dp, C.POINTER(C.c_int), dp]
        lib.fno_eom_opts_default.argtypes = [C.POINTER(EOMOpts)]
        lib.fno_eom_opts_default.restype = None
        lib.fno_eom.argtypes = [C.c_void_p, C.c_int, C.POINTER(EOMOpts), dp, dp, dp, C.POINTER(C.c_int)]
        lib.fno_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        lib.fno_get_amplitudes.argtypes = [C.c_void_p, C.c_int, dp, C.c_size_t]
        lib.fno_set_amplitudes.argtypes = [C.c_void_p, C.c_int, dp, C.c_size_t]
        lib.fno_amplitude_size.argtypes = [C.c_void_p, C.c_int]
        lib.fno_amplitude_size.restype = C.c_size_t
        lib.fno_cc_residual.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, dp]
        lib.fno_eom_size.argtypes = [C.c_void_p, C.c_int]
        lib.fno_eom_size.restype = C.c_size_t
        lib.fno_eom_sigma.argtypes = [C.c_void_p, C.c_int, C.c_int, dp, dp, C.c_size_t]
        lib.fno_eom_sigma_left.argtypes = [C.c_void_p, C.c_int, C.c_int, dp, dp, C.c_size_t]
        lib.fno_eom_vectors.argtypes = [C.c_void_p, C.c_int, C.POINTER(EOMOpts), C.c_int, dp, dp, dp,
                                        C.POINTER(C.c_int)]
        lib.fno_last_flops.argtypes = [C.c_void_p, dp, dp]
        lib.fno_last_trace.argtypes = [C.c_void_p, dp, dp, C.c_int, C.POINTER(C.c_int)]
        lib.fno_get_amplitudes_dev.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]
        lib.fno_set_amplitudes_dev.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]
        lib.fno_cc_residual_dev.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, dp]
        lib.fno_eom_sigma_dev.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_size_t]
        lib.fno_triples_residual_dev.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int] + [C.c_void_p] * 11
        lib.fno_triples_residual_dev_noalloc.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int] + [C.c_void_p] * 11
        lib.fno_dev_last_error.restype = C.c_char_p
        lib.fno_profile.argtypes = [C.c_void_p, C.c_int]
        lib.fno_profile_report.argtypes = [C.c_void_p, C.c_char_p, C.c_size_t]
        lib.fno_profile_filter.argtypes = [C.c_void_p, C.c_char_p]
        lib.fno_set_graphs.argtypes = [C.c_void_p, C.c_int]
        lib.fno_set_fused.argtypes = [C.c_void_p, C.c_int]
        lib.fno_set_autotune.argtypes = [C.c_void_p, C.c_int]
        fp = C.POINTER(C.c_float)
        lib.fno_mlp_num_params.argtypes = []
        lib.fno_mlp_num_params.restype = C.c_long
        lib.fno_mlp_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
        lib.fno_mlp_destroy.argtypes = [C.c_void_p]
        lib.fno_mlp_destroy.restype = None
        lib.fno_mlp_last_error.argtypes = [C.c_void_p]
        lib.fno_mlp_last_error.restype = C.c_char_p
        lib.fno_mlp_collect.argtypes = [C.c_void_p, C.c_void_p, C.c_long]
        lib.fno_mlp_samples.argtypes = [C.c_void_p]
        lib.fno_mlp_samples.restype = C.c_long
        lib.fno_mlp_train.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_ulong, dp]
        lib.fno_mlp_save.argtypes = [C.c_void_p, C.c_char_p]
        lib.fno_mlp_load.argtypes = [C.c_void_p, C.c_char_p]
        lib.fno_mlp_params.argtypes = [C.c_void_p, fp, C.c_size_t, C.c_int]
        lib.fno_mlp_loss_grad.argtypes = [C.c_void_p, fp, fp, C.c_long, fp, dp]
        lib.fno_mlp_predict.argtypes = [C.c_void_p, fp, C.c_long, fp]
        lib.fno_mlp_dataset.argtypes = [C.c_void_p, fp, fp, C.c_long]
        lib.fno_set_guess_model.argtypes = [C.c_void_p, C.c_void_p]
        lib.fno_last_guess_accepted.argtypes = [C.c_void_p]
        lib.fno_batch_eom.argtypes = [C.c_int, C.POINTER(C.c_void_p), C.c_int, C.POINTER(EOMOpts), dp, dp,
                                      C.POINTER(C.c_int)]
        lib.fno_batch_eom_grouped.argtypes = [C.c_int, C.POINTER(C.c_void_p), C.c_int, C.POINTER(EOMOpts), dp, dp,
                                      C.POINTER(C.c_int)]
        lib.fno_debug_tensor_size.argtypes = [C.c_void_p, C.c_char_p]
        lib.fno_debug_tensor_size.restype = C.c_size_t
        lib.fno_debug_tensor.argtypes = [C.c_void_p, C.c_char_p, dp, C.c_size_t]
        lib.fno_debug_gemm.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_long, C.c_long, C.c_long, C.c_int, C.c_int,
                                       C.c_double, C.c_double, dp, dp, dp]
        _lib = lib
    return _lib


def triples_residual_dev(device: int, nocc: int, nvir: int, prec: str, ptrs: dict, r3: int, stream: int = 0,
                         noalloc: bool = False) -> None:
    """R3 += the fused triples terms on device buffers (addresses as ints; keys of
    ptrs: T3, T2, W3_vvvv, F3_vv, W3_ovvo, W3_vvvo, W3_ovoo, W3_oooo, F3_oo)."""
    lib = library()
    fn = lib.fno_triples_residual_dev_noalloc if noalloc else lib.fno_triples_residual_dev
    names = ("T3", "T2", "W3_vvvv", "F3_vv", "W3_ovvo", "W3_vvvo", "W3_ovoo", "W3_oooo", "F3_oo")
    st = fn(device, nocc, nvir, PREC[prec], *[C.c_void_p(ptrs[k]) for k in names], C.c_void_p(r3),
            C.c_void_p(stream))
    if st != FNO_OK:
        raise FnoError(st, lib.fno_dev_last_error().decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Context:
    """One problem on one GPU: load -> [truncate] -> ccsdt -> eom."""

    def __init__(self, device: int = 0, stream=None):
        self._lib = library()
        h = C.c_void_p()
        st = self._lib.fno_create(device, C.byref(h))
        if st != FNO_OK:
            raise FnoError(st, f"fno_create failed on device {device}")
        self._h = h
        if stream is not None:
            self._check(self._lib.fno_set_stream(self._h, C.c_void_p(stream)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, allow=()):
        if st != FNO_OK and st not in allow:
            raise FnoError(st, self._lib.fno_last_error(self._h).decode())
        return st

    # ---- problem
    def load_hamiltonian(self, fock, eri, nocc: int, e_nuc: float = 0.0):
        f, g = _f64(fock), _f64(eri)
        n = f.shape[0]
        if f.shape != (n, n) or g.shape != (n, n, n, n):
            raise ValueError("fock must be (n, n) and eri (n, n, n, n)")
        self._check(self._lib.fno_load_hamiltonian(self._h, nocc, n - nocc, _dp(f), _dp(g), float(e_nuc)))

    def truncate(self, occt: float = 1.0, nvir_keep: int = 0):
        _, _, vf = self.sizes()
        kept = C.c_int()
        emp2 = C.c_double()
        occ = np.zeros(vf)
        self._check(self._lib.fno_truncate(self._h, float(occt), int(nvir_keep), C.byref(kept), C.byref(emp2),
                                           _dp(occ)))
        return kept.value, emp2.value, occ

    def mp2_energies(self):
        """(E_MP2 of the full space, E_MP2 of the truncated space) of the last truncation."""
        ef, et = C.c_double(), C.c_double()
        self._check(self._lib.fno_mp2_energies(self._h, C.byref(ef), C.byref(et)))
        return ef.value, et.value

    def xfno(self, occts, kind=None, nroots=2, cc_max_iter=100, r_tol=1e-8, e_tol=1e-10, eom_e_tol=1e-8,
             eom_r_tol=1e-6, eom_max_iter=60, allow_noconv=False):
        """fno_xfno: ground-state (and, with kind, EOM target) total energies at each
        threshold and their linear extrapolation to OCCT = 1."""
        x = np.ascontiguousarray(occts, dtype=np.float64)
        n = len(x)
        co = CCOpts()
        self._lib.fno_cc_opts_default(C.byref(co))
        co.max_iter, co.r_tol, co.e_tol = cc_max_iter, r_tol, e_tol
        eo = EOMOpts()
        self._lib.fno_eom_opts_default(C.byref(eo))
        nr = nroots if kind else 0
        eo.nroots, eo.e_tol, eo.r_tol, eo.max_iter = max(nr, 1), eom_e_tol, eom_r_tol, eom_max_iter
        kept = (C.c_int * n)()
        ecc, eeom = np.zeros(n), np.zeros(max(n * nr, 1))
        ecx, eex = C.c_double(), np.zeros(max(nr, 1))
        st = self._check(self._lib.fno_xfno(self._h, n, _dp(x), C.byref(co), KIND[kind] if kind else 0, C.byref(eo),
                                            kept, _dp(ecc), _dp(eeom), C.byref(ecx), _dp(eex)),
                         allow=(FNO_ENOCONV,) if allow_noconv else ())
        return dict(kept=list(kept), e_cc=ecc, e_eom=eeom[:n * nr].reshape(n, nr), e_cc_x=ecx.value,
                    e_eom_x=eex[:nr], converged=(st == FNO_OK))

    def sizes(self):
        o, v, vf = C.c_int(), C.c_int(), C.c_int()
        self._check(self._lib.fno_sizes(self._h, C.byref(o), C.byref(v), C.byref(vf)))
        return o.value, v.value, vf.value

    # ---- ground state
    def ccsdt(self, max_iter=100, r_tol=1e-8, e_tol=1e-10, diis_n=8, diis_start=3, prec="fp64",
              allow_noconv=False, guess=0):
        o = CCOpts()
        self._lib.fno_cc_opts_default(C.byref(o))
        o.max_iter, o.r_tol, o.e_tol, o.diis_n, o.diis_start = max_iter, r_tol, e_tol, diis_n, diis_start
        o.prec = PREC[prec]
        o.guess = guess
        ec, et, rn = C.c_double(), C.c_double(), C.c_double()
        it = C.c_int()
        st = self._check(self._lib.fno_ccsdt(self._h, C.byref(o), C.byref(ec), C.byref(et), C.byref(it),
                                             C.byref(rn)), allow=(FNO_ENOCONV,) if allow_noconv else ())
        return dict(e_corr=ec.value, e_tot=et.value, iters=it.value, res_norm=rn.value,
                    converged=(st == FNO_OK))

    def amplitude_size(self, block: int) -> int:
        return int(self._lib.fno_amplitude_size(self._h, block))

    def get_amplitudes(self, block: int) -> np.ndarray:
        out = np.zeros(self.amplitude_size(block))
        self._check(self._lib.fno_get_amplitudes(self._h, block, _dp(out), out.size))
        return out

    def set_amplitudes(self, block: int, values) -> None:
        v = _f64(values).ravel()
        self._check(self._lib.fno_set_amplitudes(self._h, block, _dp(v), v.size))

    def cc_residual(self, prec="fp64"):
        n1, n2, n3 = (self.amplitude_size(k) for k in (1, 2, 3))
        r1, r2, r3 = np.zeros(n1), np.zeros(n2), np.zeros(n3)
        ec = C.c_double()
        self._check(self._lib.fno_cc_residual(self._h, PREC[prec], _dp(r1), _dp(r2), _dp(r3), C.byref(ec)))
        return r1, r2, r3, ec.value

    def last_flops(self):
        t, a = C.c_double(), C.c_double()
        self._check(self._lib.fno_last_flops(self._h, C.byref(t), C.byref(a)))
        return t.value, a.value

    # ---- device-pointer variants: arguments are device addresses (int), e.g.
    # torch tensor .data_ptr() of contiguous float64 tensors on this device
    def set_stream(self, stream_handle) -> None:
        """Enqueue on the given HIP stream (an int handle, e.g. torch.cuda.Stream().cuda_stream)."""
        self._check(self._lib.fno_set_stream(self._h, C.c_void_p(stream_handle)))

    def set_amplitudes_dev(self, block: int, ptr: int, n: int) -> None:
        self._check(self._lib.fno_set_amplitudes_dev(self._h, block, C.c_void_p(ptr), n))

    def get_amplitudes_dev(self, block: int, ptr: int, n: int) -> None:
        self._check(self._lib.fno_get_amplitudes_dev(self._h, block, C.c_void_p(ptr), n))

    def cc_residual_dev(self, prec, p1: int, p2: int, p3: int) -> float:
        ec = C.c_double()
        self._check(self._lib.fno_cc_residual_dev(self._h, PREC[prec], C.c_void_p(p1), C.c_void_p(p2),
                                                  C.c_void_p(p3), C.byref(ec)))
        return ec.value

    def eom_sigma_dev(self, kind: str, ptr_r: int, ptr_sigma: int, n: int, prec="fp64") -> None:
        self._check(self._lib.fno_eom_sigma_dev(self._h, KIND[kind], PREC[prec], C.c_void_p(ptr_r),
                                                C.c_void_p(ptr_sigma), n))

    def last_trace(self):
        """(energies, residual norms) per iteration of the last ccsdt() call."""
        n = C.c_int()
        self._check(self._lib.fno_last_trace(self._h, None, None, 0, C.byref(n)))
        e, r = np.zeros(n.value), np.zeros(n.value)
        self._check(self._lib.fno_last_trace(self._h, _dp(e), _dp(r), n.value, C.byref(n)))
        return e, r

    # ---- profiling
    def profile(self, on: bool = True, only: str | None = None) -> None:
        """Time kernels with HIP events; `only` restricts it to names containing that text."""
        self._check(self._lib.fno_profile_filter(self._h, (only or "").encode()))
        self._check(self._lib.fno_profile(self._h, int(bool(on))))

    def set_guess_model(self, net) -> None:
        """Network used by ccsdt(guess=1); None clears it."""
        self._check(self._lib.fno_set_guess_model(self._h, None if net is None else net._h))
        self._guess_model = net  # keep it alive while the context may use it

    def last_guess_accepted(self) -> bool:
        return self._lib.fno_last_guess_accepted(self._h) == 1

    def set_autotune(self, on: bool = True) -> None:
        """Pick GEMM tiles per shape by timing every configuration on first use."""
        self._check(self._lib.fno_set_autotune(self._h, int(bool(on))))

    def set_fused(self, on: bool = True) -> None:
        """Ground-state triples residual through the fused per-triple pass (default) or per term."""
        self._check(self._lib.fno_set_fused(self._h, int(bool(on))))

    def set_graphs(self, on: bool = True) -> None:
        """Replay the residual sweep from recorded hipGraphs (default) or launch eagerly."""
        self._check(self._lib.fno_set_graphs(self._h, int(bool(on))))

    def profile_report(self) -> dict:
        import json
        size = 1 << 20
        while True:
            buf = C.create_string_buffer(size)
            st = self._lib.fno_profile_report(self._h, buf, size)
            if st == FNO_OK:
                return json.loads(buf.value.decode())
            if size > (1 << 28):
                self._check(st)
            size *= 4

    # ---- diagnostics
    def debug_tensor(self, name: str) -> np.ndarray:
        n = int(self._lib.fno_debug_tensor_size(self._h, name.encode()))
        if n == 0:
            raise KeyError(name)
        out = np.zeros(n)
        self._check(self._lib.fno_debug_tensor(self._h, name.encode(), _dp(out), n))
        return out

    def debug_gemm(self, A, B, C=None, alpha=1.0, beta=0.0, prec="fp64", tile=-1, a_kfast=True, b_nfast=True):
        """C = alpha*A@B + beta*C on the device (A: M x K, B: K x N given as logical matrices)."""
        A = _f64(A)
        B = _f64(B)
        M, K = A.shape
        N = B.shape[1]
        a = _f64(A if a_kfast else A.T)
        b = _f64(B if b_nfast else B.T)
        c = np.zeros((M, N)) if C is None else _f64(C).copy()
        self._check(self._lib.fno_debug_gemm(self._h, PREC[prec], tile, M, N, K, int(a_kfast), int(b_nfast),
                                             alpha, beta, _dp(a), _dp(b), _dp(c)))
        return c

    # ---- EOM
    def eom_size(self, kind: str) -> int:
        return int(self._lib.fno_eom_size(self._h, KIND[kind]))

    def eom_sigma(self, kind: str, r, prec="fp64") -> np.ndarray:
        x = _f64(r).ravel()
        out = np.zeros_like(x)
        self._check(self._lib.fno_eom_sigma(self._h, KIND[kind], PREC[prec], _dp(x), _dp(out), x.size))
        return out

    def eom_sigma_left(self, kind: str, l, prec="fp64") -> np.ndarray:
        """sigma^T = l^T (H-bar - E_CC) (fno_eom_sigma_left)."""
        x = _f64(l).ravel()
        out = np.zeros_like(x)
        self._check(self._lib.fno_eom_sigma_left(self._h, KIND[kind], PREC[prec], _dp(x), _dp(out), x.size))
        return out

    def eom_vectors(self, kind: str, nroots=4, left=False, max_iter=60, max_sub=0, e_tol=1e-8, r_tol=1e-6,
                    prec="fp64", allow_noconv=False, block=0):
        """Roots and right (or left) eigenvectors (fno_eom_vectors), vectors as rows."""
        o = EOMOpts()
        self._lib.fno_eom_opts_default(C.byref(o))
        o.nroots, o.max_iter, o.max_sub, o.e_tol, o.r_tol = nroots, max_iter, max_sub, e_tol, r_tol
        o.prec = PREC[prec]
        o.block = block
        dim = self.eom_size(kind)
        om, rn = np.zeros(nroots), np.zeros(nroots)
        vec = np.zeros((nroots, dim))
        it = C.c_int()
        st = self._check(self._lib.fno_eom_vectors(self._h, KIND[kind], C.byref(o), 1 if left else 0, _dp(om),
                                                   _dp(vec), _dp(rn), C.byref(it)),
                         allow=(FNO_ENOCONV,) if allow_noconv else ())
        return dict(omega=om, vectors=vec, res_norm=rn, iters=it.value, converged=(st == FNO_OK))

    def eom(self, kind: str, nroots=4, max_iter=60, max_sub=0, e_tol=1e-8, r_tol=1e-6, prec="fp64",
            allow_noconv=False, block=0):
        o = EOMOpts()
        self._lib.fno_eom_opts_default(C.byref(o))
        o.nroots, o.max_iter, o.max_sub, o.e_tol, o.r_tol = nroots, max_iter, max_sub, e_tol, r_tol
        o.prec = PREC[prec]
        o.block = block
        om, et, rn = np.zeros(nroots), np.zeros(nroots), np.zeros(nroots)
        it = C.c_int()
        st = self._check(self._lib.fno_eom(self._h, KIND[kind], C.byref(o), _dp(om), _dp(et), _dp(rn), C.byref(it)),
                         allow=(FNO_ENOCONV,) if allow_noconv else ())
        return dict(omega=om, e_tot=et, res_norm=rn, iters=it.value, converged=(st == FNO_OK))


def _fp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Mlp:
    """The learned-guess network (fno_mlp): collect samples, train, save/load, predict."""

    def __init__(self, device: int = 0):
        self._lib = library()
        h = C.c_void_p()
        st = self._lib.fno_mlp_create(device, C.byref(h))
        if st != FNO_OK:
            raise FnoError(st, f"fno_mlp_create failed on device {device}")
        self._h = h
        self.num_params = int(self._lib.fno_mlp_num_params())

    def close(self):
        if self._h is not None:
            self._lib.fno_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st != FNO_OK:
            raise FnoError(st, self._lib.fno_mlp_last_error(self._h).decode())
        return st

    def collect(self, ctx, max_samples: int = 1 << 16) -> None:
        st = self._lib.fno_mlp_collect(self._h, ctx._h, int(max_samples))
        if st != FNO_OK:
            raise FnoError(st, ctx._lib.fno_last_error(ctx._h).decode())

    @property
    def samples(self) -> int:
        return int(self._lib.fno_mlp_samples(self._h))

    def train(self, steps: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0) -> float:
        loss = C.c_double()
        self._check(self._lib.fno_mlp_train(self._h, steps, batch, lr, seed, C.byref(loss)))
        return loss.value

    def save(self, path: str) -> None:
        self._check(self._lib.fno_mlp_save(self._h, path.encode()))

    def load(self, path: str) -> None:
        self._check(self._lib.fno_mlp_load(self._h, path.encode()))

    def params(self) -> np.ndarray:
        buf = np.zeros(self.num_params, dtype=np.float32)
        self._check(self._lib.fno_mlp_params(self._h, _fp(buf), buf.size, 0))
        return buf

    def set_params(self, p) -> None:
        buf = np.ascontiguousarray(p, dtype=np.float32)
        self._check(self._lib.fno_mlp_params(self._h, _fp(buf), buf.size, 1))

    def loss_grad(self, X, T):
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        g = np.zeros(self.num_params, dtype=np.float32)
        loss = C.c_double()
        self._check(self._lib.fno_mlp_loss_grad(self._h, _fp(X), _fp(T), X.shape[0], _fp(g), C.byref(loss)))
        return loss.value, g

    def dataset(self, n: int | None = None):
        n = self.samples if n is None else n
        X = np.zeros((n, 9), dtype=np.float32)
        T = np.zeros((n, 2), dtype=np.float32)
        self._check(self._lib.fno_mlp_dataset(self._h, _fp(X), _fp(T), n))
        return X, T

    def predict(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.zeros((X.shape[0], 2), dtype=np.float32)
        self._check(self._lib.fno_mlp_predict(self._h, _fp(X), X.shape[0], _fp(Y)))
        return Y


def batch_eom(contexts, kind: str, nroots=4, max_iter=60, max_sub=0, e_tol=1e-8, r_tol=1e-6, prec="fp64",
              allow_noconv=False, block=0, grouped=False):
    """EOM roots for several contexts at once (fno_batch_eom, or fno_batch_eom_grouped with
    grouped=True); returns a list of result dicts."""
    lib = library()
    n = len(contexts)
    o = EOMOpts()
    lib.fno_eom_opts_default(C.byref(o))
    o.nroots, o.max_iter, o.max_sub, o.e_tol, o.r_tol = nroots, max_iter, max_sub, e_tol, r_tol
    o.prec = PREC[prec]
    o.block = block
    handles = (C.c_void_p * n)(*[c._h.value if isinstance(c._h, C.c_void_p) else c._h for c in contexts])
    om, rn = np.zeros(n * nroots), np.zeros(n * nroots)
    its = (C.c_int * n)()
    fn = lib.fno_batch_eom_grouped if grouped else lib.fno_batch_eom
    st = fn(n, handles, KIND[kind], C.byref(o), _dp(om), _dp(rn), its)
    if st != FNO_OK and not (allow_noconv and st == FNO_ENOCONV):
        raise FnoError(st, lib.fno_last_error(contexts[0]._h).decode())
    return [dict(omega=om[i * nroots:(i + 1) * nroots].copy(), res_norm=rn[i * nroots:(i + 1) * nroots].copy(),
                 iters=its[i], converged=(st == FNO_OK)) for i in range(n)]
