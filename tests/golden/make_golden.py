"""Write the stored expected values under tests/golden/.

Every value written here comes from the oracle's exact routines (oracle/exact_dos.py);
nothing is taken from the GPU library.  Run:  python tests/golden/make_golden.py [L ...]
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact_dos as X  # noqa: E402


def write_counts(name: str, counts: list[int], header: str) -> None:
    with open(os.path.join(HERE, name), "w") as f:
        f.write(f"# {header}\n# bin g(E)\n")
        for b, c in enumerate(counts):
            f.write(f"{b} {c}\n")


def write_lng(name: str, counts: list[int], header: str) -> None:
    lg = X.ln_g(counts)
    with open(os.path.join(HERE, name), "w") as f:
        f.write(f"# {header}\n# bin ln_g(E)   (-inf: level does not occur)\n")
        for b, v in enumerate(lg):
            f.write(f"{b} {float(v)!r}\n")


def main(argv):
    small = [("ising", 2, 4), ("potts", 3, 3)]
    for model, q, L in small:
        g = X.brute_force(model, q, L)
        write_counts(f"{model}_q{q}_L{L}_counts.txt", g,
                     f"{model} q={q} L={L} periodic: exact counts by enumeration of all states")
    for model, q, L in [("ising", 2, 6), ("ising", 2, 8), ("potts", 3, 4), ("potts", 4, 4),
                        ("potts", 3, 5), ("potts", 10, 3)]:
        g = X.transfer_matrix(model, q, L)
        write_counts(f"{model}_q{q}_L{L}_counts.txt", g,
                     f"{model} q={q} L={L} periodic: exact counts by row transfer matrix (mod-p + CRT)")
    sizes = [int(a) for a in argv] if argv else [16, 24, 32, 48, 64, 128]
    for L in sizes:
        g = X.kaufman_ising(L, processes=min(8, os.cpu_count() or 1))
        write_lng(f"ising_L{L}_lng.txt", g,
                  f"ising L={L} periodic: ln of exact counts from Kaufman's torus partition "
                  f"function (mod-p evaluation, inverse NTT, CRT); sum g = 2^N verified")


if __name__ == "__main__":
    main(sys.argv[1:])
