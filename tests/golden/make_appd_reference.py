"""Writes appd_<name>.txt: the exact magnetisation and squeezing of App. D (site-resolved form,
h = 0, local decay on every site, +x initial state) at the output times of the N = 64 open-chain
quench the benchmark integrates (alpha = 1.5, Kac-normalised J = 1, decay gamma = 0.1), every 0.1
up to t = 1.  Calls only the oracle.  Run: python tests/golden/make_appd_reference.py"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import oracle.exact as ex  # noqa: E402

CASES = {
    # name: (geometry, N, alpha, J, gamma)
    "chain64_obc_a1.5_g0.1": ("obc", 64, 1.5, 1.0, 0.1),
}


def main():
    for name, (geom, n, alpha, jscale, gamma) in CASES.items():
        J = oracle.couplings(geom, n, alpha, jscale)
        path = os.path.join(HERE, "appd_%s.txt" % name)
        with open(path, "w") as f:
            f.write("# App. D (site-resolved), %s N=%d alpha=%g J=%g gamma=%g h=0, written by "
                    "make_appd_reference.py from oracle.exact.appd_general\n" % (geom, n, alpha, jscale, gamma))
            f.write("# t Mx My Mz Cxx Cyy Czz Cxy Cxz Cyz xi2\n")
            for k in range(11):
                t = 0.1 * k
                M, C = ex.appd_general(J, gamma, t)
                x2 = ex.xi2(M, C, n) if k > 0 else 1.0
                vals = [t, *M, C[0, 0], C[1, 1], C[2, 2], C[0, 1], C[0, 2], C[1, 2], x2]
                f.write(" ".join("%.17g" % v for v in vals) + "\n")
        print(path)


if __name__ == "__main__":
    main()
