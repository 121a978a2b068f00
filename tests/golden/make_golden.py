"""Write oracle_c1.json: sampled FP64 oracle outputs for the 64^3 case.

Calls only the oracle and the input generators.  Run from the repository
root: ``python tests/golden/make_golden.py``.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2503_22139_amd import synth  # noqa: E402


def main():
    w = synth.c1()
    vol = oracle.voxelize(w.ref, w.grid, w.trunc_k)[0]
    proj = oracle.project(vol, w.grid, w.cone, w.angles)
    rng = np.random.default_rng(1234)
    vidx = rng.integers(0, vol.size, 64)
    pidx = [(int(v), int(iv), int(iu)) for v, iv, iu in
            zip(rng.integers(0, proj.shape[0], 64), rng.integers(0, proj.shape[1], 64),
                rng.integers(0, proj.shape[2], 64))]
    out = {
        "case": "c1: 4096 Gaussians, 64^3 at 1 mm, 10 views, 128x96 at 2 mm, step 0.5 mm, k=3",
        "vol_sum": float(vol.sum()),
        "proj_sum": float(proj.sum()),
        "vol_samples": [[int(i), float(vol.reshape(-1)[i])] for i in vidx],
        "proj_samples": [[list(p), float(proj[p])] for p in pidx],
    }
    with open(os.path.join(HERE, "oracle_c1.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
