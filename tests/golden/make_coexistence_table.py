"""Writes the Peng-Robinson coexistence table used by the seeded workload
generator (paper_2201_12404_amd/workloads.py, COEX_B_TABLE): Maxwell
equal-area densities (Sec. 3.1.1) of EOS set a = 0.003, b = 0.095, R = 1,
acentric factor 0.344, at T/Tc = 0.60, 0.61, ..., 0.90 and at the three
temperatures of the density ratios 1000, 100 and 10.  Calls only the oracle.

    python tests/golden/make_coexistence_table.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402


def main():
    temps = [round(0.60 + 0.01 * k, 2) for k in range(31)] + [0.592454, 0.725237, 0.901356]
    print("COEX_B_TABLE = {")
    for tr in temps:
        rv, rl, ps = O.maxwell(0.003, 0.095, 1.0, 0.344, tr)
        print(f"    {tr!r}: ({rv!r}, {rl!r}),")
    print("}")


if __name__ == "__main__":
    main()
