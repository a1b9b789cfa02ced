"""Learned-guess network and its training data, plain FP64 NumPy (test infrastructure).

Network: 9 -> 256 -> 256 -> 2 with SiLU, s(z) = z / (1 + exp(-z)), after the two
hidden layers; parameters flat in the order W1[9][256], b1, W2[256][256], b2,
W3[256][2], b3 (row-major).  Loss: mean over the batch of sum_o w_o (y_o - t_o)^2.

Features of a T3 element (i<j<k, a<b<c) and its targets:
  x / sx, |x| / sx, D / 10, e_i, e_j, e_k, e_a, e_b, e_c ;
  (t3 - x) / sx,  (fo_i + fo_j + fo_k - fv_a - fv_b - fv_c) - D
where x is the MP-style T3 guess (two Jacobi steps of the CCSDT equations from
zero amplitudes), sx its root mean square over all unique elements, D the
denominator e_i + e_j + e_k - e_a - e_b - e_c, t3 the converged amplitude and
fo/fv the diagonal of the one-body similarity-transformed Hamiltonian at the
converged amplitudes, restricted to its T1-dressed Fock part plus the T2 terms
(the dressed orbital energies of the triples equations).
"""
from __future__ import annotations

import itertools

import numpy as np

F, H, O = 9, 256, 2


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    shapes = [(F, H), (H,), (H, H), (H,), (H, O), (O,)]
    out, k = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(p[k:k + n].reshape(s))
        k += n
    assert k == p.size
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    Z1 = X @ W1 + b1
    A1 = silu(Z1)
    Z2 = A1 @ W2 + b2
    A2 = silu(Z2)
    return A2 @ W3 + b3


def loss_grad(p, X, T, w=(1.0, 1.0)):
    """Loss and flat gradient by backpropagation (chain rule written out)."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(p)
    B = X.shape[0]
    Z1 = X @ W1 + b1
    A1 = silu(Z1)
    Z2 = A1 @ W2 + b2
    A2 = silu(Z2)
    Y = A2 @ W3 + b3
    R = Y - T
    loss = float(np.sum(w * R * R) / B)
    dY = 2.0 * w * R / B
    gW3 = A2.T @ dY
    gb3 = dY.sum(0)
    dZ2 = (dY @ W3.T) * silu_grad(Z2)
    gW2 = A1.T @ dZ2
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2.T) * silu_grad(Z1)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(0)
    return loss, np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def loss_only(p, X, T, w=(1.0, 1.0)):
    Y = forward(p, np.asarray(X, dtype=np.float64))
    R = Y - np.asarray(T, dtype=np.float64)
    return float(np.sum(np.asarray(w) * R * R) / X.shape[0])


def samples(fock, eri, nocc, x3, t3, fo, fv):
    """Features and targets of every unique T3 element (row order: packed
    hole triple slow, particle triple fast, both in colex order)."""
    n = fock.shape[0]
    nvir = n - nocc
    eo, ev = np.diag(fock)[:nocc], np.diag(fock)[nocc:]

    def colex(m, g):
        return sorted(itertools.combinations(range(m), g), key=lambda t: tuple(reversed(t)))

    holes, parts = colex(nocc, 3), colex(nvir, 3)
    xs = np.array([x3[h + p] for h in holes for p in parts])
    sx = np.sqrt(np.mean(xs ** 2)) or 1.0
    X, T = [], []
    for h in holes:
        for p in parts:
            x = x3[h + p]
            D = eo[list(h)].sum() - ev[list(p)].sum()
            X.append([x / sx, abs(x) / sx, D / 10.0] + list(eo[list(h)]) + list(ev[list(p)]))
            T.append([(t3[h + p] - x) / sx, (fo[list(h)].sum() - fv[list(p)].sum()) - D])
    return np.array(X), np.array(T), sx


def dressed_hamiltonian(fock, eri, nocc, t1):
    """One- and two-body parts of e^{-T1} H e^{T1}, normal-ordered to Phi_0:
    g^ = (X x X) g (Y x Y) with X = 1 - t1 on creation slots, Y = 1 + t1 on
    annihilation slots (t1 couples occupied i with virtual a), and
    f^ = X h Y + sum_i g^[p i q i] with h = f - sum_i <p i || q i>."""
    n = fock.shape[0]
    X = np.eye(n)
    Y = np.eye(n)
    X[nocc:, :nocc] -= t1.T
    Y[nocc:, :nocc] += t1.T
    g = np.einsum("Pp,Qq,pqrs,rR,sS->PQRS", X, X, eri, Y, Y, optimize=True)
    h = fock - np.einsum("piqi->pq", eri[:, :nocc, :, :nocc])
    f = X @ h @ Y + np.einsum("piqi->pq", g[:, :nocc, :, :nocc])
    return f, g


def dressed_diagonal(fock, eri, nocc, amps):
    """fo_i = f^_ii + 1/2 sum_{n,e,f} g^[i n e f] t_in^ef,
    fv_a = f^_aa - 1/2 sum_{m,n,f} g^[m n a f] t_mn^af (the one-body diagonal
    of the triples equations at the given amplitudes).  These are the diagonals
    of the one-hole block (-fo) and the one-particle block (fv) of
    e^{-T} H e^{T} - E_CC, pinned against the determinant model with T1 and T2
    (and T3, which does not reach those blocks) in the tests."""
    o = nocc
    f, g = dressed_hamiltonian(fock, eri, o, amps[1])
    t2 = amps[2]
    fo = np.diag(f)[:o] + 0.5 * np.einsum("inef,inef->i", g[:o, :o, o:, o:], t2)
    fv = np.diag(f)[o:] - 0.5 * np.einsum("mnaf,mnaf->a", g[:o, :o, o:, o:], t2)
    return fo, fv


def mp_guess(fock, eri, nocc):
    """Two Jacobi steps of the CCSDT equations from zero amplitudes
    (t += r / D).  The first gives MP2 doubles (and no singles or triples
    for a diagonal Fock matrix); the second makes T3 = R3(T2 = MP2) / D3 and
    adds the next correction to T2."""
    from . import cc
    n = fock.shape[0]
    v = n - nocc
    amps = {1: np.zeros((nocc, v)), 2: np.zeros((nocc,) * 2 + (v,) * 2), 3: np.zeros((nocc,) * 3 + (v,) * 3)}
    D = {k: cc.denominators(fock, nocc, k, k) for k in (1, 2, 3)}
    for _ in range(2):
        R = cc.cc_residual(fock, eri, nocc, amps)
        amps = {k: amps[k] + R[k] / D[k] for k in (1, 2, 3)}
    return amps
