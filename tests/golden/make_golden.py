"""Writes the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py

heat2d_q1_16x16_F.txt : F = B K_reg^{-1} B^T (64 x 64, column-major, one value
                        per line, 17 significant digits) of the single 2D heat
                        subdomain (16x16 Q1 elements, seed of its workload),
                        long-double oracle.
elast3d_hex8_20cube_F_sample.txt : F[S, S] of subdomain 0 of the 64 x 20^3
                        hex8 elasticity workload (per-face gluing, m = 7938),
                        S = 64 columns drawn by numpy's default_rng(20) without
                        replacement, sorted; first line the indices of S, then
                        the values column-major, long-double oracle (about a
                        minute on eight cores).
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import scgen  # noqa: E402


def main():
    s = scgen.config_subdomains(1)[0]
    F = oracle.schur(s, prec="ld")
    path = os.path.join(HERE, "heat2d_q1_16x16_F.txt")
    with open(path, "w") as f:
        f.write(f"# F = B K_reg^-1 B^T, n={s.n} m={s.m}, column-major, long-double oracle\n")
        for v in F.ravel(order="F"):
            f.write(f"{v:.17g}\n")
    print("wrote", path)

    s = scgen.config_subdomains(5, count=1)[0]
    sel = np.sort(np.random.default_rng(20).choice(s.m, size=64, replace=False))
    F = oracle.schur(s, sel=sel, prec="ld")
    path = os.path.join(HERE, "elast3d_hex8_20cube_F_sample.txt")
    with open(path, "w") as f:
        f.write(f"# F[S,S] of subdomain 0, n={s.n} m={s.m}, S below, column-major, long-double oracle\n")
        f.write(" ".join(str(int(c)) for c in sel) + "\n")
        for v in F.ravel(order="F"):
            f.write(f"{v:.17g}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
