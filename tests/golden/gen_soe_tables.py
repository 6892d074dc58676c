"""Write the SOE tables used by the tests (tests/golden/soe_talbot_M*.txt).

Calls only the oracle's fitter (oracle.soe.best_talbot_soe): a midpoint rule on
Weideman's Talbot contour for the inverse-Laplace representation of the
Gaussian (Sec. 3 of the paper).  Both the oracle and the GPU library take these
tables as an input parameter of the method.

Run from the repository root:  python tests/golden/gen_soe_tables.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import soe  # noqa: E402


def main():
    for M in (8, 12, 16, 20, 24):
        w, s, err = soe.best_talbot_soe(M)
        path = os.path.join(HERE, "soe_talbot_M%d.txt" % M)
        with open(path, "w") as f:
            f.write("# SOE of exp(-x^2): sum_l w_l exp(-s_l |x|), M = %d terms\n" % M)
            f.write("# Talbot-contour midpoint rule (oracle.soe.best_talbot_soe)\n")
            f.write("# sup |error| on [0, 200] = %.3e\n" % err)
            f.write("# Re(w) Im(w) Re(s) Im(s)\n")
            for wl, sl in zip(w, s):
                f.write("%.17e %.17e %.17e %.17e\n" % (wl.real, wl.imag, sl.real, sl.imag))
        print(path, err)


if __name__ == "__main__":
    main()
