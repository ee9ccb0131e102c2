"""Writes tests/golden/ggq16_oracle.txt: the oracle's own 16-node near-panel
rules (Sec. 3.1), built by oracle.ggq.table().  Run from the repository root:
    python tests/golden/make_ggq_golden.py
"""
import os
import sys
import warnings

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ggq  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ggq16_oracle.txt")


def main():
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        tab = ggq.table()
    with open(OUT, "w") as f:
        f.write("# 16-node near-panel rules built by oracle/ggq.py (node elimination, Sec. 3.1)\n")
        f.write("# block name, then 16 rows [target Gauss-Legendre index] of 16 values [node]\n")
        for name in ("self_x", "self_w", "right_x", "right_w"):
            f.write(name + "\n")
            for row in tab[name]:
                f.write(" ".join(repr(float(v)) for v in row) + "\n")


def load(path=OUT):
    import numpy as np
    out, cur = {}, None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        if line[0].isalpha():
            cur = line.strip()
            out[cur] = []
        else:
            out[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in out.items()}


if __name__ == "__main__":
    main()
