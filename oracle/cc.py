"""Spin-orbital CCSDT and EOM-CCSDT in FP64 on the CPU (test infrastructure).

Part of the oracle: used only by tests, the smoke check and the CPU
baseline; it shares no code with the GPU library.

* Residuals and energy: eqs (5)-(6), evaluated term by term by the Wick
  expansion in ``oracle.wick`` (no factorisation beyond pairwise einsum).
* EOM sigma vectors: eqs (1)-(4) for IP (1h, 2h1p, 3h2p), DIP (2h, 3h1p,
  4h2p), EA (1p, 2p1h, 3p2h) and DEA (2p, 3p1h, 4p2h), sigma = <mu|(H-bar R)_C|0>,
  eigenvalues omega = E_target - E_CC.
* Solvers (the paper names none): Jacobi updates t += r / D with
  D = sum f_holes - sum f_particles, DIIS on the update vectors, and a
  block Davidson for the right EOM eigenvectors.  Norms and DIIS products
  run over unique amplitudes (i<j<..., a<b<...).

Dense arrays hold every amplitude rank: t1[i,a], t2[i,j,a,b], t3[i,j,k,a,b,c];
R blocks likewise r[h..., p...].
"""
from __future__ import annotations

import math

import numpy as np

from . import wick


# ---------------------------------------------------------------- helpers
def reference_energy(fock, eri, nocc, e_nuc=0.0) -> float:
    """<Phi_0|H|Phi_0> = sum_i f_ii - 1/2 sum_ij <ij||ij> (+ nuclear repulsion)."""
    o = slice(0, nocc)
    return float(np.trace(fock[o, o]) - 0.5 * np.einsum("ijij->", eri[o, o, o, o]) + e_nuc)


def denominators(fock, nocc, nh, np_):
    """D = sum_holes f_hh - sum_particles f_pp as a dense array over [h..., p...]."""
    eo = np.diag(fock)[:nocc]
    ev = np.diag(fock)[nocc:]
    d = np.zeros((nocc,) * nh + (len(ev),) * np_)
    for k in range(nh):
        shape = [1] * (nh + np_)
        shape[k] = nocc
        d = d + eo.reshape(shape)
    for k in range(np_):
        shape = [1] * (nh + np_)
        shape[nh + k] = len(ev)
        d = d - ev.reshape(shape)
    return d


def unique_mask(nocc, nvir, nh, np_):
    """Boolean mask of the unique elements (strictly increasing holes and particles)."""
    m = np.ones((nocc,) * nh + (nvir,) * np_, dtype=bool)
    for k in range(nh - 1):
        idx = np.arange(nocc)
        s1 = [1] * (nh + np_)
        s2 = [1] * (nh + np_)
        s1[k] = nocc
        s2[k + 1] = nocc
        m &= idx.reshape(s1) < idx.reshape(s2)
    for k in range(np_ - 1):
        idx = np.arange(nvir)
        s1 = [1] * (nh + np_)
        s2 = [1] * (nh + np_)
        s1[nh + k] = nvir
        s2[nh + k + 1] = nvir
        m &= idx.reshape(s1) < idx.reshape(s2)
    return m


def _tensors(fock, eri, nocc, amps):
    T = wick.Tensors(fock, eri, nocc)
    for k, t in amps.items():
        T.amps[("t", k, k)] = t
    return T


_MERGED = {}


def _merged_cc(k):
    if k not in _MERGED:
        _MERGED[k] = wick.merge_external(wick.cc_terms(k), k, k)
    return _MERGED[k]


def _merged_eom(mu, nu):
    key = ("eom", mu, nu)
    if key not in _MERGED:
        _MERGED[key] = wick.merge_external(wick.eom_terms(mu, nu), mu[0], mu[1])
    return _MERGED[key]


# ---------------------------------------------------------------- CC
def cc_energy(fock, eri, nocc, amps) -> float:
    """Correlation energy, eq (6) minus E_ref."""
    T = _tensors(fock, eri, nocc, amps)
    return float(wick.evaluate(wick.cc_terms(0), T, ()))


def cc_residual(fock, eri, nocc, amps, ranks=(1, 2, 3)):
    """Dense residuals r_k = <Phi_k| e^{-T} H e^{T} |Phi_0>, eq (5)."""
    nvir = fock.shape[0] - nocc
    T = _tensors(fock, eri, nocc, amps)
    out = {}
    for k in ranks:
        terms, G = _merged_cc(k)
        shape = (nocc,) * k + (nvir,) * k
        out[k] = wick.antisymmetrize(wick.evaluate(terms, T, shape), k, k) / G
    return out


def cc_residual_element(fock, eri, nocc, amps, k, index) -> float:
    """One residual element <Phi_mu|e^{-T}He^{T}|Phi_0> (unmerged classes, no dense output)."""
    T = _tensors(fock, eri, nocc, amps)
    return float(wick.evaluate(wick.cc_terms(k), T, None, fixed=tuple(index)))


def _udot(a, b, nocc, nvir, rank_pairs):
    s = 0.0
    for key, (nh, np_) in rank_pairs.items():
        w = 1.0 / (math.factorial(nh) * math.factorial(np_))
        s += w * float(np.vdot(a[key], b[key]))
    return s


class CCResult(dict):
    pass


def solve_ccsdt(fock, eri, nocc, ranks=(1, 2, 3), max_iter=100, r_tol=1e-10, e_tol=1e-12,
                diis_n=8, diis_start=3, amps0=None, e_nuc=0.0, callback=None):
    """Jacobi + DIIS solution of eq (5); returns energies, amplitudes and history."""
    nvir = fock.shape[0] - nocc
    D = {k: denominators(fock, nocc, k, k) for k in ranks}
    amps = {k: np.zeros((nocc,) * k + (nvir,) * k) for k in ranks}
    if amps0:
        for k, t in amps0.items():
            amps[k] = t.copy()
    rp = {k: (k, k) for k in ranks}
    e_ref = reference_energy(fock, eri, nocc, e_nuc)
    e_old = cc_energy(fock, eri, nocc, amps)
    hist_t, hist_e = [], []
    history = []
    converged = False
    rnorm = float("inf")
    it = 0
    for it in range(1, max_iter + 1):
        R = cc_residual(fock, eri, nocc, amps, ranks)
        rnorm = math.sqrt(_udot(R, R, nocc, nvir, rp))
        new = {k: amps[k] + R[k] / D[k] for k in ranks}
        err = {k: new[k] - amps[k] for k in ranks}
        hist_t.append(new)
        hist_e.append(err)
        if len(hist_t) > diis_n:
            hist_t.pop(0)
            hist_e.pop(0)
        if diis_n > 0 and it >= diis_start and len(hist_t) >= 2:
            m = len(hist_t)
            B = -np.ones((m + 1, m + 1))
            B[m, m] = 0.0
            for a in range(m):
                for b in range(a, m):
                    B[a, b] = B[b, a] = _udot(hist_e[a], hist_e[b], nocc, nvir, rp)
            scale = max(abs(B[a, a]) for a in range(m))
            if scale > 0:
                B[:m, :m] /= scale
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            c = np.linalg.lstsq(B, rhs, rcond=None)[0][:m]
            new = {k: sum(c[a] * hist_t[a][k] for a in range(m)) for k in ranks}
        amps = new
        e = cc_energy(fock, eri, nocc, amps)
        de = e - e_old
        e_old = e
        history.append((it, e, rnorm, de))
        if callback:
            callback(it, e, rnorm, de)
        if rnorm < r_tol and abs(de) < e_tol:
            converged = True
            break
    return CCResult(e_corr=e_old, e_tot=e_old + e_ref, e_ref=e_ref, amps=amps, iters=it,
                    res_norm=rnorm, converged=converged, history=history)


# ---------------------------------------------------------------- EOM
EOM_SPACES = wick.EOM_SPACES


def eom_sigma(fock, eri, nocc, amps, kind, rblocks, mu_blocks=None):
    """sigma_mu = <Phi_mu| (H_N e^T R)_C |Phi_0> for every block mu of the ``kind`` R space."""
    nvir = fock.shape[0] - nocc
    _, blocks = EOM_SPACES[kind]
    T = _tensors(fock, eri, nocc, amps)
    out = {}
    for mu in (mu_blocks or blocks):
        shape = (nocc,) * mu[0] + (nvir,) * mu[1]
        acc = np.zeros(shape)
        for nu in blocks:
            if nu not in rblocks:
                continue
            T.amps[("r",) + nu] = rblocks[nu]
            terms, G = _merged_eom(mu, nu)
            acc += wick.evaluate(terms, T, shape) / G
            del T.amps[("r",) + nu]
        out[mu] = wick.antisymmetrize(acc, mu[0], mu[1])
    return out


def eom_sigma_element(fock, eri, nocc, amps, kind, rblocks, mu, index) -> float:
    """One element of sigma_mu (unmerged classes, externals fixed; amplitudes may be lazy arrays)."""
    _, blocks = EOM_SPACES[kind]
    T = _tensors(fock, eri, nocc, amps)
    val = 0.0
    for nu in blocks:
        if nu not in rblocks:
            continue
        T.amps[("r",) + nu] = rblocks[nu]
        val += float(wick.evaluate(wick.eom_terms(mu, nu), T, None, fixed=tuple(index)))
        del T.amps[("r",) + nu]
    return val


def eom_diagonal(fock, nocc, kind):
    """Zeroth-order diagonal sum f_particles - sum f_holes for each R block."""
    _, blocks = EOM_SPACES[kind]
    return {b: -denominators(fock, nocc, b[0], b[1]) for b in blocks}


class _Space:
    """Unique-element vector layout of an R space (concatenated blocks)."""

    def __init__(self, nocc, nvir, blocks):
        self.blocks = blocks
        self.masks = {b: unique_mask(nocc, nvir, *b) for b in blocks}
        self.sizes = {b: int(self.masks[b].sum()) for b in blocks}
        self.dim = sum(self.sizes.values())
        self.nocc, self.nvir = nocc, nvir

    def pack(self, d):
        return np.concatenate([d[b][self.masks[b]] for b in self.blocks])

    def unpack(self, x):
        out = {}
        off = 0
        for b in self.blocks:
            arr = np.zeros(self.masks[b].shape)
            arr[self.masks[b]] = x[off:off + self.sizes[b]]
            out[b] = wick.antisymmetrize(arr, b[0], b[1])
            off += self.sizes[b]
        return out


def eom_matrix(fock, eri, nocc, amps, kind):
    """Explicit EOM matrix over unique elements (column j = sigma of unit vector j)."""
    nvir = fock.shape[0] - nocc
    _, blocks = EOM_SPACES[kind]
    sp = _Space(nocc, nvir, [b for b in blocks])
    M = np.zeros((sp.dim, sp.dim))
    for j in range(sp.dim):
        e = np.zeros(sp.dim)
        e[j] = 1.0
        M[:, j] = sp.pack(eom_sigma(fock, eri, nocc, amps, kind, sp.unpack(e)))
    return M, sp


def eom_sigma_left(fock, eri, nocc, amps, kind, lblocks):
    """Left-hand sigma l^T (H-bar - E_CC) over unique elements: the transpose of
    the EOM matrix (columns = sigma of unit vectors) applied to l, as blocks."""
    M, sp = eom_matrix(fock, eri, nocc, amps, kind)
    return sp.unpack(M.T @ sp.pack(lblocks))


def eom_left_dense(fock, eri, nocc, amps, kind, nroots):
    """Lowest ``nroots`` eigenvalues (by real part) of the explicit EOM matrix and
    its left eigenvectors (columns l with l^T M = w l^T, unit 2-norm), as blocks."""
    M, sp = eom_matrix(fock, eri, nocc, amps, kind)
    w, Lv = np.linalg.eig(M.T)
    order = np.argsort(w.real)[:nroots]
    return w[order], [sp.unpack(np.real(Lv[:, j]) / np.linalg.norm(np.real(Lv[:, j]))) for j in order], M, sp


def eom_roots_dense(fock, eri, nocc, amps, kind, nroots):
    """Lowest ``nroots`` eigenvalues (by real part) of the explicit EOM matrix."""
    M, sp = eom_matrix(fock, eri, nocc, amps, kind)
    w = np.linalg.eigvals(M)
    w = w[np.argsort(w.real)]
    return w[:nroots], M, sp


def davidson(fock, eri, nocc, amps, kind, nroots, max_iter=60, max_sub=None, e_tol=1e-9,
             r_tol=1e-6, nguess=None, callback=None):
    """Block Davidson for the lowest right EOM eigenpairs (real parts).

    Guesses: unit vectors on the lowest zeroth-order diagonal entries of the
    principal (first) block, continued into the other blocks (lowest diagonal
    first) when the principal block has fewer entries than roots.  Preconditioner (theta - D)^-1 with D the
    zeroth-order diagonal over all blocks.  Orthonormalisation: classical
    Gram-Schmidt applied twice.
    """
    nvir = fock.shape[0] - nocc
    _, blocks = EOM_SPACES[kind]
    sp = _Space(nocc, nvir, list(blocks))
    diag = sp.pack(eom_diagonal(fock, nocc, kind))
    max_sub = max_sub or 8 * nroots
    nguess = nguess or nroots
    first = sp.sizes[blocks[0]]
    order = list(np.argsort(diag[:first], kind="stable"))
    order += [first + int(j) for j in np.argsort(diag[first:], kind="stable")]
    order = order[:nguess]
    V = np.zeros((sp.dim, 0))
    for j in order:
        e = np.zeros(sp.dim)
        e[j] = 1.0
        V = np.column_stack([V, e])
    S = np.zeros((sp.dim, 0))
    theta_old = np.full(nroots, np.inf)
    history = []
    conv = False
    for it in range(1, max_iter + 1):
        k0 = S.shape[1]
        newS = [sp.pack(eom_sigma(fock, eri, nocc, amps, kind, sp.unpack(V[:, j])))
                for j in range(k0, V.shape[1])]
        S = np.column_stack([S] + newS) if newS else S
        G = V.T @ S
        w, Y = np.linalg.eig(G)
        idx = np.argsort(w.real)[:nroots]
        theta = w[idx].real
        Yr = Y[:, idx].real
        X = V @ Yr
        nrm = np.linalg.norm(X, axis=0)
        X /= nrm
        Yr /= nrm
        Rr = S @ Yr - X * theta
        rn = np.linalg.norm(Rr, axis=0)
        de = np.abs(theta - theta_old)
        history.append((it, theta.copy(), rn.copy()))
        if callback:
            callback(it, theta, rn)
        theta_old = theta
        if np.all(rn < r_tol) and np.all(de < e_tol):
            conv = True
            break
        if V.shape[1] + nroots > max_sub:
            V, _ = np.linalg.qr(X)
            S = np.zeros((sp.dim, 0))
            continue
        add = []
        for j in range(nroots):
            if rn[j] < r_tol:
                continue
            den = theta[j] - diag
            den = np.where(np.abs(den) < 1e-8, 1e-8, den)
            d = Rr[:, j] / den
            for _ in range(2):
                d -= V @ (V.T @ d)
                for a in add:
                    d -= a * (a @ d)
            n = np.linalg.norm(d)
            if n > 1e-10:
                add.append(d / n)
        if not add:
            conv = True
            break
        V = np.column_stack([V] + add)
    return dict(omega=theta, res_norm=rn, iters=it, converged=conv, history=history,
                vectors=X, space=sp)
