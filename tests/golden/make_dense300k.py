"""Write dense300k_trajectory.json: the FP64 oracle's registration of the
dense 300k RGB-D frame pair (TEST INFRASTRUCTURE; calls only the oracle and
the input generator).

Workload: synth.rgbd_pair(300000, 300000, seed=3, select="random") (a seeded
random subset of 300,000 valid pixels of each synthetic 640x480 frame),
cutoff 3 ell, ell = 0.2 * 0.25**(s/3) over 4 stages of 25 iterations, the
fixed step tau = ell^2 / F, a^2 = mean |x_i|^2, b^2 = 1, T0 = I.  Each
iteration's F, omega, v (eq. scalar, eq. 3_gradient) is summed over every
pair inside the cutoff, enumerated through the oracle's grid (the brute-force
pair set).  Stored per iteration: the oracle's trace row (F, omega, v, tau,
ell, pairs, pose after the step) and the sums of |terms| that scale the
tolerance of omega and v.

Run from the repository root: python tests/golden/make_dense300k.py
(about 15 minutes on 8 cores).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1904_02266_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dense300k_trajectory.json")


def inputs():
    p = synth.rgbd_pair(300000, 300000, seed=3, select="random")
    return p


def input_digest(p):
    h = hashlib.sha256()
    for a in (p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    p = inputs()
    ells = [0.2 * 0.25 ** (s / 3.0) for s in range(4)]
    t0 = time.time()
    r = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, kappa=3.0, stage_iters=(25, 25, 25),
                        stage_ell=ells, max_iters=100, grid=True)
    assert r["rc"] == 0 and r["iters"] == 100, r["rc"]
    doc = {
        "workload": "rgbd_pair(300000, 300000, seed=3, select='random'); kappa 3; ell 0.2*0.25**(s/3), "
                    "4 x 25 iterations; fixed step tau = ell^2/F; a2 = mean|x|^2; b2 = 1; T0 = I",
        "input_sha256": input_digest(p),
        "a2": oracle.mean_sqnorm(p.src_xyz),
        "stage_ell": ells,
        "trace": r["trace"].tolist(),
        "abs": r["abs"].tolist(),
        "oracle_seconds": time.time() - t0,
        "threads": oracle.default_threads(),
    }
    with open(OUT, "w") as f:
        json.dump(doc, f)
    print(OUT, f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
