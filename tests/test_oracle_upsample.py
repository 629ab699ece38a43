"""Pins of the oracle's coarse-medium upsampling (trilinear samples of a coarse node grid
at the simulation nodes, both grids spanning the same box): exact on fields linear in
x, y, z; the identity when the grids coincide; coarse node values reproduced where fine
nodes coincide with them; every value a convex combination of its eight coarse nodes;
and a brute-force per-node evaluation."""
import numpy as np

import oracle


def test_linear_fields_exact():
    mz, my, mx = 5, 4, 7
    z, y, x = np.meshgrid(np.linspace(0, 1, mz), np.linspace(0, 1, my), np.linspace(0, 1, mx), indexing="ij")
    f = 3.0 + 2.0 * x - 1.5 * y + 0.25 * z
    nx, ny, nz = 19, 11, 9
    Z, Y, X = np.meshgrid(np.linspace(0, 1, nz), np.linspace(0, 1, ny), np.linspace(0, 1, nx), indexing="ij")
    want = 3.0 + 2.0 * X - 1.5 * Y + 0.25 * Z
    np.testing.assert_allclose(oracle.upsample(f, (nx, ny, nz)), want, rtol=0, atol=1e-13)


def test_identity_and_coincident_nodes():
    rng = np.random.default_rng(5)
    c = rng.random((4, 5, 6))
    np.testing.assert_array_equal(oracle.upsample(c, (6, 5, 4)), c)
    # (n - 1) a multiple of (m - 1): every coarse node is a fine node
    f = oracle.upsample(c, (11, 9, 7))
    np.testing.assert_allclose(f[::2, ::2, ::2], c, rtol=0, atol=1e-15)


def test_convex_combination_and_brute_force():
    rng = np.random.default_rng(6)
    c = rng.random((3, 4, 5)) * 100.0
    shape = (13, 7, 8)
    f = oracle.upsample(c, shape)
    nx, ny, nz = shape
    mz, my, mx = c.shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                q = (i * (mx - 1) / (nx - 1), j * (my - 1) / (ny - 1), k * (mz - 1) / (nz - 1))
                lo = [min(int(np.floor(qq)), m - 2) for qq, m in zip(q, (mx, my, mz))]
                t = [qq - l for qq, l in zip(q, lo)]
                v = 0.0
                corners = []
                for a in (0, 1):
                    for b in (0, 1):
                        for d in (0, 1):
                            w = (t[0] if a else 1 - t[0]) * (t[1] if b else 1 - t[1]) * (t[2] if d else 1 - t[2])
                            val = c[lo[2] + d, lo[1] + b, lo[0] + a]
                            v += w * val
                            corners.append(val)
                assert abs(f[k, j, i] - v) <= 1e-12 * abs(v)
                assert min(corners) - 1e-12 <= f[k, j, i] <= max(corners) + 1e-12
