"""Small test utilities (random antisymmetric amplitudes); no method arithmetic."""
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
