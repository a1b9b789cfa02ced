"""Host unit tests of the library's small dense solvers (csrc/linalg.cpp).

The solvers are compiled on the CPU with g++ and the address and
undefined-behaviour sanitizers (tests/linalg_check.cpp drives them) and
compared with LAPACK through numpy: eigenvalues of nonsymmetric matrices
(Hessenberg reduction + Francis double-shift QR), the symmetric
eigenproblem, linear solves and inverse iteration.  The Davidson solver uses
these on its subspace matrices, so the cases include matrices of that kind
(diagonally dominant, nonsymmetric) besides the classic hard ones (cyclic
permutations, complex pairs, repeated eigenvalues).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "paper_2509_14157_amd", "csrc", "linalg.cpp")
DRIVER = os.path.join(HERE, "linalg_check.cpp")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("linalg") / "linalg_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", DRIVER, SRC, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def run(exe, lines):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout.splitlines()


def fmt(a):
    return " ".join(repr(float(x)) for x in np.ravel(a))


def match_multiset(got, ref, tol):
    got = list(got)
    for z in ref:
        k = int(np.argmin([abs(g - z) for g in got]))
        assert abs(got[k] - z) <= tol, (z, got[k], tol)
        got.pop(k)


def eig_cases():
    rng = np.random.default_rng(7)
    cases = []
    for n in (1, 2, 3, 4, 5, 8, 13, 32, 64):
        cases.append(rng.standard_normal((n, n)))
    # Davidson-like subspace matrices: diagonal-dominant, mildly nonsymmetric
    for n in (16, 48, 96):
        d = np.sort(rng.uniform(0.2, 3.0, n))
        a = np.diag(d) + 0.05 * rng.standard_normal((n, n))
        cases.append(a)
    # cyclic permutations: |eigenvalues| all 1, standard shifts stall
    for n in (3, 4, 6):
        cases.append(np.roll(np.eye(n), 1, axis=0))
    # rotation blocks: complex pairs
    q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    blk = np.zeros((6, 6))
    for k, (r, w) in enumerate([(1.0, 2.0), (-0.5, 0.3), (2.0, 1e-3)]):
        blk[2 * k:2 * k + 2, 2 * k:2 * k + 2] = [[r, w], [-w, r]]
    cases.append(q @ blk @ q.T)
    # repeated eigenvalues (diagonalizable), already triangular, zero, tiny scale
    s = rng.standard_normal((7, 7))
    cases.append(s @ np.diag([1, 1, 1, 2, 2, -3, 0.0]) @ np.linalg.inv(s))
    cases.append(np.triu(rng.standard_normal((9, 9))))
    cases.append(np.zeros((5, 5)))
    cases.append(1e-200 * rng.standard_normal((6, 6)))
    cases.append(1e150 * rng.standard_normal((6, 6)))
    return cases


def test_nonsym_eigvals_match_lapack(exe):
    cases = eig_cases()
    out = run(exe, [f"eig {a.shape[0]} {fmt(a)}" for a in cases])
    assert len(out) == len(cases)
    for a, line in zip(cases, out):
        assert line != "fail", a
        v = np.array(line.split(), dtype=float).reshape(-1, 2)
        got = v[:, 0] + 1j * v[:, 1]
        ref = np.linalg.eigvals(a)
        scale = max(np.abs(a).max(), np.finfo(float).tiny)
        # repeated eigenvalues of a non-normal matrix are sensitive: sqrt(eps)
        tol = 1e-6 * scale if a.shape[0] == 7 else 1e-9 * scale * max(1, a.shape[0])
        match_multiset(got, ref, tol)
        # conjugate pairs come out as pairs with exactly opposite imaginary parts
        for k in np.nonzero(v[:, 1] > 0)[0]:
            assert k + 1 < len(v) and v[k + 1, 1] == -v[k, 1] and v[k + 1, 0] == v[k, 0]


def test_sym_eig_matches_lapack(exe):
    rng = np.random.default_rng(3)
    cases = []
    for n in (1, 2, 5, 17, 40):
        x = rng.standard_normal((n, n))
        cases.append(x + x.T)
    cases.append(np.diag([3.0, 1.0, 1.0, -2.0]))  # degenerate, already diagonal
    out = run(exe, [f"sym {a.shape[0]} {fmt(a)}" for a in cases])
    for a, line in zip(cases, out):
        n = a.shape[0]
        v = np.array(line.split(), dtype=float)
        w, vec = v[:n], v[n:].reshape(n, n)
        np.testing.assert_allclose(w, np.linalg.eigvalsh(a), atol=1e-12 * max(1, np.abs(a).max()))
        assert np.all(np.diff(w) >= 0)
        np.testing.assert_allclose(vec.T @ vec, np.eye(n), atol=1e-12)
        np.testing.assert_allclose(a @ vec, vec * w, atol=1e-11 * max(1, np.abs(a).max()))


def test_solve_and_singular(exe):
    rng = np.random.default_rng(5)
    a = rng.standard_normal((12, 12))
    b = rng.standard_normal(12)
    sing = np.ones((3, 3))
    out = run(exe, [f"solve 12 {fmt(a)} {fmt(b)}", f"solve 3 {fmt(sing)} 1 2 3"])
    np.testing.assert_allclose(np.array(out[0].split(), dtype=float), np.linalg.solve(a, b), rtol=1e-10, atol=1e-12)
    assert out[1] == "singular"


def test_inverse_iteration_gives_eigenvector(exe):
    rng = np.random.default_rng(11)
    n = 20
    a = np.diag(np.linspace(0.5, 4.0, n)) + 0.05 * rng.standard_normal((n, n))
    lams = np.linalg.eigvals(a)
    lams = np.sort(lams[np.abs(lams.imag) < 1e-12].real)[:3]
    out = run(exe, [f"inv {n} {float(lam)!r} {fmt(a)}" for lam in lams])
    for lam, line in zip(lams, out):
        x = np.array(line.split(), dtype=float)
        assert abs(np.linalg.norm(x) - 1) < 1e-12
        assert np.linalg.norm(a @ x - lam * x) < 1e-8
