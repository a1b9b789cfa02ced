"""Write synthetic_sha256.json: SHA-256 of the seeded generator's output bytes.

Run from the repository root: ``python tests/golden/make_synthetic_hashes.py``.
The hashes pin the input recipe (PCG64 seed, draw order, symmetrisation) so
that the CPU oracle and the GPU library are known to consume identical bytes.
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from synthetic import make_hamiltonian  # noqa: E402

CASES = [(3, 5, 7, 0.3, 3.0), (4, 12, 1, 0.3, 3.0), (10, 60, 2, 0.2, 6.0), (6, 20, 400, 0.3, 3.0)]

if __name__ == "__main__":
    out = {}
    for o, v, seed, lo, hi in CASES:
        out[f"{o},{v},{seed},{lo},{hi}"] = make_hamiltonian(o, v, seed, evir=(lo, hi)).sha256()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synthetic_sha256.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)
