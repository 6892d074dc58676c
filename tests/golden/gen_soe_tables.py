"""Write the SOE tables used by the tests (tests/golden/soe_*_M*.txt).

Calls only the oracle's fitters: oracle.soe.best_talbot_soe (a midpoint rule on
Weideman's Talbot contour for the inverse-Laplace representation of the
Gaussian, Sec. 3 of the paper) and oracle.soe.reduced_soe (balanced truncation
of a long Talbot table, the model reduction behind the paper's VPMR tables).  Both the oracle and the GPU library take these
tables as an input parameter of the method.

Run from the repository root:  python tests/golden/gen_soe_tables.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import soe  # noqa: E402


def write(path, M, how, w, s, err):
    with open(path, "w") as f:
        f.write("# SOE of exp(-x^2): sum_l w_l exp(-s_l |x|), M = %d terms\n" % M)
        f.write("# %s\n" % how)
        f.write("# sup |error| on [0, 200] = %.3e\n" % err)
        f.write("# Re(w) Im(w) Re(s) Im(s)\n")
        for wl, sl in zip(w, s):
            f.write("%.17e %.17e %.17e %.17e\n" % (wl.real, wl.imag, sl.real, sl.imag))
    print(path, err)


def main():
    for M in (8, 12, 16, 20, 24):
        w, s, err = soe.best_talbot_soe(M)
        write(os.path.join(HERE, "soe_talbot_M%d.txt" % M), M,
              "Talbot-contour midpoint rule (oracle.soe.best_talbot_soe)", w, s, err)
    for M in (10,):
        w, s, err = soe.reduced_soe(M)
        write(os.path.join(HERE, "soe_reduced_M%d.txt" % M), M,
              "balanced truncation of the 48-term Talbot table + minimax polish "
              "(oracle.soe.reduced_soe)", w, s, err)


if __name__ == "__main__":
    main()
