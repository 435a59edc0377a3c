"""Writes sampler_vectors.json from the oracle's sampler alone.

The C++ sampler of the library is checked against these vectors; the
oracle's sampler is itself pinned by the published SplitMix64 vector, the
Lemire power-of-two identity and the exhaustive Fisher-Yates enumeration.
Run: python tests/golden/make_sampler_vectors.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.sampler import SplitMix64, bounded, sample_landmarks  # noqa: E402

CASES = [
    (1, 1, 0), (10, 10, 5), (10, 3, 0), (100, 7, 42), (5000, 200, 0),
    (5000, 200, 1), (5000, 200, 2), (1_000_000, 1000, 0), (1_000_000, 2000, 7),
    (1_000_000, 4000, 123456789), (2**40, 16, 2**63 + 12345), (3000, 2999, 3),
]


def main():
    out = {"sample_landmarks": [], "bounded": []}
    for n, l, seed in CASES:
        out["sample_landmarks"].append(
            {"n": n, "l": l, "seed": str(seed), "idx": sample_landmarks(n, l, seed)})
    for seed, k in [(7, 3), (7, 1000), (9, 2**63 + 1), (11, 2**64 - 1), (13, 6)]:
        g = SplitMix64(seed)
        out["bounded"].append({"seed": str(seed), "k": str(k),
                               "draws": [str(bounded(g, k)) for _ in range(20)]})
    with open(os.path.join(HERE, "sampler_vectors.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
