"""Write taus_lift_streams.txt: for seed 1234, the first stream index whose raw seed word for each
Tausworthe component lies below 2^(32-k) (k = 31, 29, 28), i.e. a stream whose seeding needs the
lift.  Oracle only; about a minute.

    python tests/golden/make_taus_lift_streams.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle as orc  # noqa: E402

if __name__ == "__main__":
    lines = ["# seed component stream raw_word  (first stream whose raw word i is below 2^(32-k))",
             "# written by tests/golden/make_taus_lift_streams.py"]
    for comp, k in ((0, 31), (1, 29), (2, 28)):
        j = orc.find_small_seed_word(1234, comp, 1 << (32 - k))
        w = orc.seed_word(1234, j, comp)
        print(comp, j, w, flush=True)
        lines.append("1234 %d %d %d" % (comp, j, w))
    with open(os.path.join(HERE, "taus_lift_streams.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
