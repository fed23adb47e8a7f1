"""Writes peps_d16_fingerprint.txt: projections of the full-size fermionic
PEPS double layer E = A^dagger o A (U(1) x fZ2, D = 16, interleaved to rank
8 with the Koszul sign of the interleave; sections "Fermionic tensor
networks" and "Adjoint") onto seeded random +-1 vectors, computed by the
blockwise CPU oracle over every block of E.  Inputs: A filled with small
integers, so every entry of E and every projection is an exact integer in
fp64 and the stored values are independent of summation order.

Calls only oracle/ (and the seeded input generators).  Runs for about ten
minutes on 8 cores:  python tests/golden/make_peps_d16_fingerprint.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import blockwise  # noqa: E402
from oracle.graded import Space, Structure  # noqa: E402
from paper_2508_10076_amd import synth  # noqa: E402

NPROJ = 4


def main():
    cfg = synth.config5()
    tA, call = cfg["tensors"]["A"], cfg["call"]
    osp = lambda s: Space(s.sectors, s.degs, s.dual)
    stA = Structure(tA["sym"], [osp(s) for s in tA["cod"]], [osp(s) for s in tA["dom"]])
    a = synth.small_ints(stA.size, 5, 16)
    stAd, bAd = blockwise.adjoint(stA, stA.to_blocks(a))
    ad = stAd.from_blocks(bAd)
    stE, e = blockwise.contract_storage(stAd, ad, call["pA"], call["qA"], stA, a, call["pB"], call["qB"],
                                        call["pAB"], call["qAB"])
    lines = ["# E = A^dagger o A, config D=16 (1,2,2,2,1), A = synth.small_ints(nnz(A), 5, 16)",
             "# written by tests/golden/make_peps_d16_fingerprint.py (blockwise CPU oracle, every block)",
             f"size {stE.size}",
             f"nonzero {int(np.count_nonzero(e))}",
             f"sum_sq {float(np.dot(e, e)):.1f}"]
    for k in range(NPROJ):
        w = synth.signs(stE.size, 5, k)
        lines.append(f"proj{k} {float(np.dot(w, e)):.1f}")
    with open(os.path.join(HERE, "peps_d16_fingerprint.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
