"""Writes tests/golden/fig1_shape.txt.  Calls only the oracle package.

Sec. 3.1 / Fig. 1 describe five inputs hashed into a range of ten, where one
value (3) appears twice and shares its bucket with a different value (10121).
The figure's hash values are not in the text, so this script searches for the
smallest seed under which 3 and 10121 share a bucket for V = 10, adds two more
inputs that land elsewhere, and stores the oracle's table for that input.
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402


def main():
    V = 10
    seed = 0
    while oracle.bucket_one(3, V, seed) != oracle.bucket_one(10121, V, seed):
        seed += 1
    b3 = oracle.bucket_one(3, V, seed)
    extra = []
    x = 100
    while len(extra) < 2:
        if oracle.bucket_one(x, V, seed) != b3 and all(
                oracle.bucket_one(x, V, seed) != oracle.bucket_one(e, V, seed) for e in extra):
            extra.append(x)
        x += 1
    keys = np.array([3, extra[0], 10121, 3, extra[1]], np.uint32)
    off, ids, _ = oracle.build_table(keys, V, seed)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fig1_shape.txt")
    with open(out, "w") as f:
        f.write("# written by tests/golden/make_golden.py from the oracle; see its docstring\n")
        f.write("keys=%s\n" % ",".join(str(int(k)) for k in keys))
        f.write("V=%d\nseed=%d\n" % (V, seed))
        f.write("offsets=%s\n" % ",".join(str(int(v)) for v in off))
        f.write("ids=%s\n" % ",".join(str(int(v)) for v in ids))
    print(open(out).read())


if __name__ == "__main__":
    main()
