"""Pins of the damping profile and the printed stability constant."""
import json
import math
import os

import numpy as np

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_cerjan_edge_value_and_shape():
    g = GOLD["cerjan_edge"]
    nb = g["width"]
    cfg = oracle.Config((64, 50, 40), 10.0, 1e-3, 1, sponge=(nb,) * 6, alpha=g["alpha"])
    p = oracle.profiles(cfg)
    assert abs(p[(0, 0)][0] - g["edge_factor"]) < 1e-15
    assert abs(p[(0, 0)][-1] - g["edge_factor"]) < 1e-15
    # default coefficient 0.3 / width reproduces the 20-cell value
    p2 = oracle.profiles(oracle.Config((64, 50, 40), 10.0, 1e-3, 1, sponge=(nb,) * 6))
    assert abs(p2[(1, 0)][0] - g["edge_factor"]) < 1e-15
    for (ax, half), prof in p.items():
        n = cfg.shape[ax]
        last = n - 1 - half
        core = prof[: last + 1]
        # symmetric about the grid centre at the sample's own coordinate
        assert np.allclose(core, core[::-1], rtol=0, atol=1e-15)
        # 1 in the interior, < 1 inside the zone, non-decreasing towards the interior
        assert np.all(core[nb: last + 1 - nb] == 1.0)
        assert np.all(core[:nb] < 1.0)
        assert np.all(np.diff(core[: n // 2]) >= 0.0)


def test_free_surface_drops_top_sponge():
    cfg = oracle.Config((30, 30, 30), 10.0, 1e-3, 1, sponge=(8,) * 6, free_surface=True)
    p = oracle.profiles(cfg)
    assert p[(2, 0)][0] == 1.0 and p[(2, 1)][0] == 1.0
    assert p[(2, 0)][-1] < 1.0


def test_printed_cfl_constant_near_von_neumann_bound():
    """Eq.(5) prints 0.495; the exact 3D O(2,4) bound is 1/(sqrt(3) (9/8 + 1/24))."""
    c1 = GOLD["eq4_stencil"]["coeff_half"]
    c2 = GOLD["eq4_stencil"]["coeff_three_halves"]
    bound = 1.0 / (math.sqrt(3.0) * (abs(c1) + abs(c2)))
    assert abs(bound - 6.0 / (7.0 * math.sqrt(3.0))) < 1e-15
    printed = GOLD["eq5_cfl"]["factor"]
    assert 0.0 < printed - bound < 1e-3  # the printed value is the bound rounded up
