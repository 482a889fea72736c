"""Writes the stored expected values under tests/golden/.  Calls only the
oracle package (its LP formulation solved by HiGHS) and the input generator."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle.lp as lp  # noqa: E402
from paper_2602_22421_amd.instances import config_instance  # noqa: E402


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    inst = config_instance(0)
    opt, eta = lp.sblp(inst)
    with open(os.path.join(here, "config0_lp.txt"), "w") as f:
        f.write("# LP optimum of the sales-based LP (GAM form of eqs. 5-9) for the\n")
        f.write("# L=1000, n=50, A=I workload (seed 0), solved by HiGHS through oracle.lp.\n")
        f.write(f"opt {opt!r}\n")
        f.write("eta " + " ".join(repr(float(x)) for x in eta) + "\n")


if __name__ == "__main__":
    main()
