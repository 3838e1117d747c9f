"""The seeded input generators shared by the oracle and the GPU path:
deterministic, with the stated distributions and mesh recipes."""
import numpy as np

from paper_1512_02390_amd import workloads as W


def test_generators_are_deterministic_and_distinct_per_seed():
    shape = (33, 41)
    for gen in (W.random_guess, W.random_nodal):
        a, b = gen(shape, W.BC_DIRICHLET, 7), gen(shape, W.BC_DIRICHLET, 7)
        assert np.array_equal(a, b)
        assert not np.array_equal(a, gen(shape, W.BC_DIRICHLET, 8))


def test_generator_ranges_and_boundary():
    shape = (65, 65)
    u = W.random_guess(shape, W.BC_DIRICHLET, 3)
    f = W.random_nodal(shape, W.BC_DIRICHLET, 3)
    inner = (slice(1, -1), slice(1, -1))
    assert u[inner].min() >= 0.0 and u[inner].max() < 1.0
    assert f[inner].min() >= -1.0 and f[inner].max() < 1.0
    # i.i.d. uniform: means 1/2 and 0 within a few standard errors
    n = u[inner].size
    assert abs(u[inner].mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(f[inner].mean()) < 5 * np.sqrt(1 / 3 / n)
    for a in (u, f):
        assert not a[0].any() and not a[-1].any() and not a[:, 0].any() and not a[:, -1].any()
    # periodic arrays keep every entry
    assert np.all(W.random_guess((8, 8), W.BC_PERIODIC, 3) > 0.0)


def test_workload_meshes():
    c4, c5 = W.config("c4"), W.config("c5")
    for cfg, n in ((c4, 32), (c5, 48)):
        h = np.diff(cfg.xb)
        assert len(h) == n and abs(cfg.xb[0]) == 0.0
        assert abs(h[0] - 1.0 / n) < 1e-15 and abs(h[-1] / h[0] - 16.0) < 1e-12   # aspect ratio 1 -> 16
        assert np.all(np.diff(h) > 0)
        assert np.allclose(cfg.yb, np.linspace(0.0, 1.0, n + 1))
    assert W.node_array_shape(64, 64, 8, W.BC_DIRICHLET) == (513, 513)      # 511^2 unknowns
    assert W.node_array_shape(128, 128, 16, W.BC_DIRICHLET) == (2049, 2049)
    assert W.node_array_shape(4, 4, 6, W.BC_PERIODIC) == (24, 24)


def test_random_field_grid_evaluation_matches_pointwise():
    """The tensor-grid fast path of GaussianFieldNu equals the per-node
    evaluation of the same random Fourier features (rounding only)."""
    import numpy as np
    from paper_1512_02390_amd import workloads as W
    f = W.GaussianFieldNu(ell=0.1)
    x = np.linspace(0.0, 1.0, 37)
    y = np.linspace(-0.3, 1.2, 29)
    grid = W.nodal(f.nu, x, y)
    X, Y = np.meshgrid(x, y)
    point = np.array([f.nu(a, b) for a, b in zip(X.ravel(), Y.ravel())]).reshape(X.shape)
    assert np.abs(grid - point).max() <= 1e-13 * np.abs(point).max()
