"""Write the FP64 oracle's reference for the 1024x1024x24 GAP-ITV2D workload at
its full iteration count (200 outer x 10 inner FGP, lambda = 0.1): PSNR of x
and theta against the truth, global sums of x, and full rows of x and theta
at fixed (frame, row) positions. The GPU parity test compares its own solve
with these sampled values. Inputs come from the seeded generator; Y is formed
by the oracle. Only the oracle computes anything here.

Run from the repository root:  python tests/golden/make_cacti_reference.py
(about 10 minutes on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2005_08028_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cacti_1024x24_gap_itv2d_200x10.json")
X_ROWS = [(k, i) for k in (0, 12, 23) for i in (0, 511, 1023)]
THETA_ROWS = [(k, i) for k in (0, 23) for i in (256, 767)]


def main():
    c = synth.CONFIGS["cacti_1024x24"]
    pr = synth.problem_from_config("cacti_1024x24")
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    lam = float(np.float32(c["lam"]))
    t0 = time.time()
    x, th = orc.gap_tv(Y, pr.masks, lam, c["T"], c["N"], tv=c["tv"])
    secs = time.time() - t0
    ref = {
        "about": "FP64 oracle reference for GAP-ITV2D on the 1024x1024x24 CACTI-style workload (seed 3, shifted "
                 "Bernoulli(0.5) masks, texture N(0, 0.02^2)), 200 outer x 10 inner FGP iterations, lambda = 0.1 "
                 "(as float32), written by tests/golden/make_cacti_reference.py from the oracle alone.",
        "workload": "cacti_1024x24", "tv": c["tv"], "lam": lam, "T": c["T"], "N": c["N"],
        "oracle_seconds": round(secs, 1),
        "psnr_x": orc.psnr(x, pr.truth), "psnr_theta": orc.psnr(th, pr.truth),
        "sum_x": float(x.sum()), "sumsq_x": float((x * x).sum()),
        "x_rows": [{"frame": k, "row": i, "values": [float("%.12g" % v) for v in x[k, i]]} for k, i in X_ROWS],
        "theta_rows": [{"frame": k, "row": i, "values": [float("%.12g" % v) for v in th[k, i]]}
                       for k, i in THETA_ROWS],
    }
    with open(OUT, "w") as f:
        json.dump(ref, f)
    print(f"wrote {OUT}: PSNR x {ref['psnr_x']:.4f} dB, {secs:.0f} s")


if __name__ == "__main__":
    main()
