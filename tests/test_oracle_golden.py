"""Regression guard: the oracle still reproduces its stored 64^3 outputs."""
import json
import os

import numpy as np

import oracle
from paper_2503_22139_amd import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_c1_regression():
    with open(os.path.join(HERE, "oracle_c1.json")) as f:
        g = json.load(f)
    w = synth.c1()
    vol = oracle.voxelize(w.ref, w.grid, w.trunc_k)[0]
    proj = oracle.project(vol, w.grid, w.cone, w.angles)
    assert abs(vol.sum() - g["vol_sum"]) <= 1e-12 * abs(g["vol_sum"])
    assert abs(proj.sum() - g["proj_sum"]) <= 1e-12 * abs(g["proj_sum"])
    flat = vol.reshape(-1)
    for i, v in g["vol_samples"]:
        assert abs(flat[i] - v) <= 1e-13 * max(1.0, abs(v))
    for p, v in g["proj_samples"]:
        assert abs(proj[tuple(p)] - v) <= 1e-12 * max(1.0, abs(v))
