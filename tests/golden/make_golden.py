"""Write the stored expected values under tests/golden/ from the CPU oracle only.

    python tests/golden/make_golden.py config2     # n = 16, d = 0.70, 2000 FP64 iterations

Each output file states the oracle calls that produced it.  Nothing here touches
the GPU library.
"""
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle.native as on  # noqa: E402
from oracle import bdc  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
LN2 = math.log(2.0)


def config2(n=16, d=0.70, iters=2000, checkpoints=(0, 1, 10, 100, 500, 1000, 2000)):
    """FP64 BA (Section 2.3) on the oracle's CSR channel from the uniform law,
    log p floored at 700 nats below its max (the library's FP64 iteration rule);
    records the Blahut bounds of the iterate after each checkpoint."""
    csr = on.CSR(n)
    lp = bdc.uniform_logp(n)
    rows = []
    t0 = time.time()
    for t in range(iters + 1):
        D, L, U, I, _ = csr.evaluate(d, lp, floor_nats=700.0)
        if t in checkpoints:
            rows.append((t, L / LN2, U / LN2, I / LN2, float(np.min(bdc.normalise_logp(lp)))))
            print("t=%d L=%.15f U=%.15f (%.0f s)" % (t, L / LN2, U / LN2, time.time() - t0), flush=True)
        if t == iters:
            break
        lp = bdc.floor_logp(bdc.normalise_logp(lp) + D - L, 700.0)
    path = os.path.join(HERE, "config2_n16_d070.txt")
    with open(path, "w") as f:
        f.write("# BA iterates for the binary deletion channel, n = %d, d = %.2f, FP64, p0 uniform.\n" % (n, d))
        f.write("# Written by tests/golden/make_golden.py config2 from oracle.native.CSR.evaluate\n")
        f.write("# (brute-force counts, Section 2.3 iteration, log p floored at max - 700 nats).\n")
        f.write("# columns: iteration t, lower bound L (bits), upper bound U (bits), I(p_t) (bits), min log p_t\n")
        for r in rows:
            f.write("%d %.17g %.17g %.17g %.17g\n" % r)
    print("wrote", path)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "config2"
    if which == "config2":
        config2()
    else:
        raise SystemExit("unknown target " + which)
