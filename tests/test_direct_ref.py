"""Pins the sampled direct-sum gradient helper to the oracle's direct gradient."""
import numpy as np

import oracle as O
from direct_ref import direct_grad_at
from paper_1305_1825_amd import workloads as W


def test_closed_form_direct_gradient_matches_oracle_with_images():
    c = W.config_colloid_10k(n=300, p=2)
    P = c["params"]
    gr, gq = O.direct_grad(P, c["x"], c["y"], c["z"], c["q"])
    idx = W.sample_indices(300, 25, tag=5)
    sr, sq = direct_grad_at(P, c["x"], c["y"], c["z"], c["q"], idx)
    scale_r = np.sqrt(np.mean(gr ** 2))
    scale_q = np.sqrt(np.mean(gq ** 2))
    assert np.max(np.abs(sr - gr[idx])) <= 1e-12 * scale_r
    assert np.max(np.abs(sq - gq[idx])) <= 1e-12 * scale_q


def test_closed_form_direct_gradient_matches_oracle_in_cube():
    c = W.config_cube_1k(n=200)
    P = c["params"]
    gr, gq = O.direct_grad(P, c["x"], c["y"], c["z"], c["q"])
    idx = np.arange(0, 200, 7)
    sr, sq = direct_grad_at(P, c["x"], c["y"], c["z"], c["q"], idx)
    assert np.max(np.abs(sr - gr[idx])) <= 1e-12 * np.sqrt(np.mean(gr ** 2))
    assert np.max(np.abs(sq - gq[idx])) <= 1e-12 * np.sqrt(np.mean(gq ** 2))
