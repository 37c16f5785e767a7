"""Write lf_primitivity.txt: irreducibility (hence primitivity, the degrees being Mersenne
exponents) of every lagged-Fibonacci trinomial x^ll + x^sl + 1 of Table I, computed by the oracle
only.  The largest row takes tens of minutes on one core.

    python tests/golden/make_lf_primitivity.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle as orc  # noqa: E402

PAIRS = [(2281, 1252), (4423, 3004), (9689, 5502), (19937, 10095), (23209, 12470), (23209, 13470),
         (44497, 23463), (132049, 54454), (756839, 279695), (859433, 288477), (3021377, 1010202)]

if __name__ == "__main__":
    lines = ["# Table I trinomials x^ll + x^sl + 1: ll sl primitive|reducible",
             "# written by tests/golden/make_lf_primitivity.py (oracle.trinomial_irreducible, Rabin's test)"]
    for ll, sl in PAIRS:
        t = time.time()
        ok = orc.trinomial_irreducible(ll, sl)
        print(ll, sl, ok, "%.1fs" % (time.time() - t), flush=True)
        lines.append("%d %d %s" % (ll, sl, "primitive" if ok else "reducible"))
    with open(os.path.join(HERE, "lf_primitivity.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
