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


# ------------------------------------------------------------------ coarse medium read in the scheme
#
# With Config.coarse the oracle reads every medium value as a trilinear sample of the coarse
# grid at the value's own position: rho at the velocity samples, lambda and mu at the nodes,
# mu at the shear samples (the paper's textures read with trilinear filtering).  The set-up
# reading instead samples the coarse grid at the simulation nodes once (upsample) and then
# takes the node means.

STAG = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0, 0), (0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)]


def _positions(shape, q):
    """True coordinates (x, y, z) in grid units of the samples of medium array q."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = STAG[q]
    return x + s[0], y + s[1], z + s[2]


def _active(shape, q):
    nx, ny, nz = shape
    x, y, z = _positions(shape, q)
    return (x <= nx - 1) & (y <= ny - 1) & (z <= nz - 1)


def _both(shape, cshape, lam_c, mu_c, rho_c):
    cfg_c = oracle.Config(shape, 10.0, 1e-3, 1, coarse=cshape)
    cfg_n = oracle.Config(shape, 10.0, 1e-3, 1)
    coarse = oracle.medium(cfg_c, lam_c, mu_c, rho_c)
    setup = oracle.medium(cfg_n, *(oracle.upsample(a, shape) for a in (lam_c, mu_c, rho_c)))
    return coarse, setup


def test_coarse_reading_exact_on_linear_fields():
    """A medium linear in x, y, z: the coarse reading returns the linear function at every
    sample's own (staggered) position, and so does the set-up reading."""
    shape, cshape = (23, 17, 13), (6, 5, 4)
    mx, my, mz = cshape
    nx, ny, nz = shape
    Zc, Yc, Xc = np.meshgrid(np.arange(mz), np.arange(my), np.arange(mx), indexing="ij")
    # coefficients per fine grid unit: coarse coordinate X = x (m - 1) / (n - 1)
    lin = lambda a, b, c, d: (a + b * Xc * (nx - 1) / (mx - 1) + c * Yc * (ny - 1) / (my - 1)
                              + d * Zc * (nz - 1) / (mz - 1))
    coefs = {"lam": (7e9, 2e7, -1e7, 3e7), "mu": (5e9, -1e7, 4e7, 2e7), "rho": (2500.0, 3.0, -2.0, 5.0)}
    fields = {k: lin(*v) for k, v in coefs.items()}
    coarse, setup = _both(shape, cshape, fields["lam"], fields["mu"], fields["rho"])
    arr = ["rho", "rho", "rho", "lam", "mu", "mu", "mu", "mu"]
    for q in range(8):
        a, b, c, d = coefs[arr[q]]
        x, y, z = _positions(shape, q)
        m = _active(shape, q)
        want = a + b * x + c * y + d * z
        np.testing.assert_allclose(coarse[q][m], want[m], rtol=1e-13, atol=0)
        np.testing.assert_allclose(setup[q][m], want[m], rtol=1e-13, atol=0)
        assert not coarse[q][~m].any()


def test_coarse_reading_on_the_simulation_grid_is_the_node_reading():
    """A coarse grid equal to the simulation grid: the samples at half positions are the
    node means the scheme takes for node arrays."""
    rng = np.random.default_rng(21)
    shape = (9, 8, 7)
    c = [2e9 + 1e9 * rng.random((7, 8, 9)) for _ in range(2)] + [2000.0 + 500.0 * rng.random((7, 8, 9))]
    coarse = oracle.medium(oracle.Config(shape, 10.0, 1e-3, 1, coarse=shape), *c)
    node = oracle.medium(oracle.Config(shape, 10.0, 1e-3, 1), *c)
    np.testing.assert_allclose(coarse, node, rtol=1e-15, atol=0)


def test_coarse_reading_differs_only_where_a_mean_straddles_a_coarse_node():
    """Random coarse medium: the coarse reading and the set-up reading agree (1e-13) at
    the nodes and at every half position whose two nodes lie in one coarse cell along each
    half axis; where a coarse node lies strictly between them the two differ (the
    piecewise-linear samples have a kink there), by at most the coarse field's second
    difference."""
    rng = np.random.default_rng(22)
    shape, cshape = (29, 22, 18), (7, 6, 5)  # (n - 1)/(m - 1) not an integer on any axis
    nx, ny, nz = shape
    mx, my, mz = cshape
    lam_c, mu_c = (3e9 + 2e9 * rng.random((mz, my, mx)) for _ in range(2))
    rho_c = 2000.0 + 800.0 * rng.random((mz, my, mx))
    coarse, setup = _both(shape, cshape, lam_c, mu_c, rho_c)
    n, m = np.array(shape), np.array(cshape)

    def straddles(ax, lo):
        """A coarse node strictly between the coarse coordinates of fine nodes lo, lo + 1."""
        X0, X1 = lo * (m[ax] - 1) / (n[ax] - 1), (lo + 1) * (m[ax] - 1) / (n[ax] - 1)
        return np.floor(X0) + 1.0 < X1

    any_diff = 0
    for q in range(8):
        x, y, z = _positions(shape, q)
        act = _active(shape, q)
        strad = np.zeros(act.shape, dtype=bool)
        for ax, p in enumerate((x, y, z)):
            if STAG[q][ax]:
                strad |= straddles(ax, np.floor(p))
        scale = np.abs(setup[q][act]).max()
        same = act & ~strad
        np.testing.assert_allclose(coarse[q][same], setup[q][same], rtol=0, atol=1e-13 * scale)
        diff = np.abs(coarse[q] - setup[q])[act & strad]
        if q in (3, 4):
            assert not (act & strad).any()  # nodes have no mean
        else:
            assert diff.size > 0 and (diff > 1e-9 * scale).mean() > 0.5, q
            any_diff += diff.size
            # |difference| <= the largest jump of the coarse field (a loose second-difference bound)
            arr = rho_c if q < 3 else mu_c
            assert diff.max() <= np.ptp(arr), q
    assert any_diff > 0
