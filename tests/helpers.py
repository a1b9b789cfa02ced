"""Small test utilities (random antisymmetric amplitudes, device buffers); no method arithmetic."""
import itertools
import math

import numpy as np


def perm_sign(p):
    p = list(p)
    s = 1
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


def random_antisym(rng, nocc, nvir, nh, np_, scale):
    """Random array over [h..., p...] antisymmetric in the holes and in the particles."""
    shape = (nocc,) * nh + (nvir,) * np_
    x = rng.normal(0.0, scale, shape)
    out = np.zeros(shape)
    for ph in itertools.permutations(range(nh)):
        for pp in itertools.permutations(range(np_)):
            perm = list(ph) + [nh + q for q in pp]
            out += perm_sign(ph) * perm_sign(pp) * x.transpose(perm)
    return out / math.sqrt(math.factorial(nh) * math.factorial(np_))


def random_amps(rng, nocc, nvir, scales=(0.1, 0.05, 0.03)):
    return {k: random_antisym(rng, nocc, nvir, k, k, s) for k, s in zip((1, 2, 3), scales)}


class HipBuffers:
    """Device buffers and a stream from the HIP runtime the library itself
    loaded (torch 2.10+rocm7.0 bundles a second HIP runtime with the same
    SONAME; two runtimes in one process do not share devices or streams, so
    the caller-side memory here comes from the library's runtime)."""

    def __init__(self):
        import ctypes
        self.C = ctypes
        self.lib = ctypes.CDLL("libamdhip64.so.7")
        self.bufs = []

    def _ok(self, st):
        assert st == 0, st

    def alloc(self, n):
        p = self.C.c_void_p()
        self._ok(self.lib.hipMalloc(self.C.byref(p), self.C.c_size_t(8 * max(n, 1))))
        self.bufs.append(p)
        return p.value

    def upload(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        p = self.alloc(x.size)
        self._ok(self.lib.hipMemcpy(self.C.c_void_p(p), x.ctypes.data_as(self.C.c_void_p),
                                    self.C.c_size_t(8 * x.size), 1))
        return p

    def download(self, p, n):
        out = np.zeros(n)
        self._ok(self.lib.hipMemcpy(out.ctypes.data_as(self.C.c_void_p), self.C.c_void_p(p), self.C.c_size_t(8 * n),
                                    2))
        return out

    def stream(self):
        s = self.C.c_void_p()
        self._ok(self.lib.hipStreamCreate(self.C.byref(s)))
        return s.value

    def sync(self, s):
        self._ok(self.lib.hipStreamSynchronize(self.C.c_void_p(s)))

    def close(self, s):
        self._ok(self.lib.hipStreamDestroy(self.C.c_void_p(s)))
        for p in self.bufs:
            self._ok(self.lib.hipFree(p))
