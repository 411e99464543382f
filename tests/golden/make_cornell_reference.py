"""Writes cornell64_d5_mean.json: the image mean of the Cornell box (64 x 64
pixels, max depth 5, jittered pinhole camera) from a 65,536 spp render of
the CPU oracle with every count equal to one (a plain path tracer with
BSDF sampling and NEE under the balance heuristic; MARS is unbiased for any
counts, supplement A.1), per channel, with its standard error.

    python tests/golden/make_cornell_reference.py

It calls only oracle/ (the renderer under test never writes a stored value)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import scenegen  # noqa: E402
from oracle import oracle as orc  # noqa: E402

ITERS, SPP = 256, 256


def main():
    sc = scenegen.make_cornell(64, 64)
    o = orc.Oracle(sc, max_depth=5)
    o.set_fixed_beta(np.array([[1.0, 1.0, 0.0]]))
    means = []
    for i in range(ITERS):
        o.render_iteration(orc.Oracle.params(iteration=50000 + i, spp=SPP, alloc=orc.ALLOC_FIXED))
        means.append(o.sample_radiance().astype(np.float64).mean(0))
    m = np.array(means)
    out = {"scene": "cornell 64x64, max depth 5, seed 1 (scenegen.make_cornell)",
           "counts": "fixed (1, 1): BSDF and NEE, balance heuristic, no Russian roulette",
           "spp": ITERS * SPP, "iterations": ITERS, "first_iteration": 50000,
           "mean_rgb": m.mean(0).tolist(),
           "stderr_rgb": (m.std(0, ddof=1) / np.sqrt(ITERS)).tolist(),
           "source": "oracle/ only (tests/golden/make_cornell_reference.py)"}
    with open(os.path.join(HERE, "cornell64_d5_mean.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
