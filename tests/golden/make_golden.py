"""Write tests/golden/oracle_outputs.json from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py
The digests pin the oracle to itself across changes (the paper prints no
test vectors); every value comes from oracle.shuffle of arange(n).
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

CASES = [
    # (n, seed, rounds)
    (1, 0, 24), (5, 1, 24), (16, 3, 24), (17, 3, 24), (100, 42, 24),
    (100_000, 42, 4),  # the small single-shuffle workload: 4 rounds, domain 2^17
    (100_000, 42, 24), (65_537, 7, 24), (65_536, 7, 24), (123_457, 0xFFFFFFFFFFFFFFFF, 16),
]


def main():
    cases = []
    for n, seed, rounds in CASES:
        out = oracle.shuffle(np.arange(n, dtype=np.uint32), seed, rounds)
        cases.append({"n": n, "seed": seed, "rounds": rounds,
                      "sha256": hashlib.sha256(out.tobytes()).hexdigest(),
                      "head": out[:16].tolist()})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_outputs.json")
    with open(path, "w") as fh:
        json.dump({"generator": "tests/golden/make_golden.py (oracle only)",
                   "payload": "arange(n) as uint32", "cases": cases}, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
