"""Writes the stored expected values under tests/golden/ by calling only the
oracle (oracle/).  Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def hash_vectors():
    rng = np.random.default_rng(20230605)
    rows = []
    edge = [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF, 0x9E3779B9]
    pairs = [(a, b) for a in edge for b in edge]
    pairs += [(int(a), int(b)) for a, b in rng.integers(0, 2**32, (220, 2), dtype=np.uint64)]
    for h, w in pairs:
        rows.append(f"step {h:08x} {w:08x} {oracle.hash_step(h, w):08x}")
    for _ in range(400):
        seed = int(rng.integers(0, 2**32))
        l = int(rng.integers(-300, 300))
        k = int(rng.integers(0, 5))
        m = int(rng.integers(0, 2 ** (k + 1))) if k else 0
        i, j = (int(x) for x in rng.integers(-2**30, 2**30, 2))
        ai, aj = (int(x) for x in rng.integers(-16384, 16384, 2))
        s = int(rng.integers(0, 2))
        rows.append(f"texel {seed:08x} {l} {k} {m} {i} {j} {ai} {aj} {s} "
                    f"{oracle.texel_hash(seed, l, k, m, i, j, ai, aj, s):08x}")
    with open(os.path.join(HERE, "hash_vectors.txt"), "w") as f:
        f.write("# hash test vectors written by tests/golden/make_golden.py from the FP64 oracle\n")
        f.write("# step h w -> H(h,w) = fmix32((h^w)+0x9E3779B9) (MurmurHash3 finaliser)\n")
        f.write("# texel seed l k m i j ai aj s -> hash of one per-texel random number\n")
        f.write("\n".join(rows) + "\n")


if __name__ == "__main__":
    hash_vectors()
