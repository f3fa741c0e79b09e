"""Host-side checks of the coarse-to-fine grid rebuild: the product's cube
grid (torch, here on the CPU) has the tet indexing of the input generator's
grid and the vertex coordinates the oracle defines, and the rebuilt cube is
the oracle's."""
import numpy as np
import torch

import synth
from oracle import coarse as ocoarse
from paper_2406_01579_amd import coarse


def test_grid_matches_generator_and_oracle():
    R = 5
    low, h = np.array([-0.7, -0.2, 0.05], np.float32), np.float32(0.23)
    v, t = coarse.kuhn_grid(R, low, h, device="cpu")
    _, t_ref = synth.kuhn_grid(R)
    assert np.array_equal(t.numpy(), t_ref.astype(np.int32))
    assert np.array_equal(v.numpy(), ocoarse.grid_vertices(low, h, R))


def test_resized_cube_matches_oracle():
    lo, hi = np.array([-0.31, -0.2, 0.1], np.float32), np.array([0.4, 0.27, 0.33], np.float32)
    a = coarse.resized_cube(lo, hi, 32, 2.0 / 32)
    b = ocoarse.resized_cube(lo, hi, 32, 2.0 / 32)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
