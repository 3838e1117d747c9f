"""The learned Schwarz parameters end to end on the GPU: training data from
the solver's own sweeps, training with the library's kernels, the network's
per-element parameters consumed by the Schwarz kernels (checked against the
oracle), and the gain of the trained network over the paper's parameters
(ceil(p_l/8) overlap, full transition width) on the 32 x 32 stretched
variable-diffusion workload, where both converge, measured in iterations and
as the cost per decade of residual reduction omega = W / r_bar of the full
MGCG solve to 1e-10."""
import math

import numpy as np
import pytest

from paper_1512_02390_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def trained():
    from paper_1512_02390_amd import learned
    patches = learned.default_patches(ars=(1.0, 4.0, 16.0), sigmas=(0.0, 1.0), ps=(12,))
    print(f"[gpu-learned] sweep of {len(patches)} patches", flush=True)
    X, T, recs = learned.make_dataset(patches)
    for pt, rows, lab in recs:
        best = min(rows, key=lambda t: t[3])
        print(f"  AR {pt.ar:4.0f} sigma {pt.sigma} p {pt.p}: label alpha {lab[0]:.2f} "
              f"rho {lab[1] / 2:.3f} (r_bar {best[2]:.2f}, omega {best[3]:.1f})", flush=True)
    net, hist = learned.train(X, T, steps=1500)
    print(f"  training loss {hist[0]:.3e} -> {hist[-1]:.3e}", flush=True)
    yield learned, net, X, T, hist
    net.close()


def test_training_fits_the_labels(trained):
    learned, net, X, T, hist = trained
    assert hist[-1] < hist[0]
    err = (net.forward(X) - T).abs().max().item()
    print(f"  max label error {err:.3f}")
    assert err < 0.2


def _problem():
    """The 32 x 32 stretched variable-diffusion workload (aspect ratio 1 to 16,
    nu = exp(g), p = 12): the paper's parameters converge there, so the
    comparison is between two converging solves."""
    cfg = W.config("c4")
    return cfg.xb, cfg.yb, cfg.p


def _solve(s, fn, kind="mg11"):
    """(iterations, converged, omega, overlaps) of the MGCG solve to 1e-10;
    only a non-finite residual (SEM_ENAN) counts as no reduction."""
    from paper_1512_02390_amd import learned
    from paper_1512_02390_amd.sem import SemError
    shape = s.shape()
    b = s.zeros()
    s.mass(torch.tensor(fn, dtype=torch.float64, device="cuda"), b)
    u = torch.tensor(W.random_guess(shape, 0, W.SEED_U0), dtype=torch.float64, device="cuda")
    ns1, ns2 = learned.schedule(s.L, kind)
    ov = [0] + [s.level_info(l)[1] for l in range(1, s.L + 1)]
    try:
        it, hist, ok = s.pcg_solve(u, b, 300, 1e-10, ns1, ns2)
    except SemError as e:
        if e.status != -6:
            raise
        return 300, False, math.inf, ov
    w = learned.cycle_cost(s.p, ov, [a + c for a, c in zip(ns1, ns2)])
    return it, ok, w / learned.rbar(hist), ov


def test_learned_parameters_beat_the_paper_on_the_workload(trained):
    """Iterations of the full solve to 1e-10 (and the cost per decade
    omega = W / r_bar, reported): the trained network's parameters, reduced
    per level (the learned solver's default), against the paper's on the same
    problem, both converging; the per-element mode is solved and reported
    beside them (its W from the largest overlap per level, an upper bound)."""
    from paper_1512_02390_amd.sem import Solver
    learned, net, *_ = trained
    xb, yb, p = _problem()
    NU = learned.nodal_nu(xb, yb, p, 0, W.GaussianFieldNu())
    fn = W.random_nodal(NU.shape, 0, W.SEED_RHS)
    paper = Solver(xb, yb, p, 0, 1, 1, 5, nu=NU)
    it_p, ok_p, om_p, ov_p = _solve(paper, fn)
    paper.close()
    out = {}
    for mode in ("level", "element"):
        s, ep = learned.solver_with_learned(xb, yb, p, 0, NU, net, mode=mode)
        assert ep is not None
        out[mode] = _solve(s, fn)
        s.close()
        it_l, ok_l, om_l, ov_l = out[mode]
        print(f"  learned ({mode}): overlaps {ov_l[1:]}, alpha {ep[:, 0].min():.2f}.."
              f"{ep[:, 0].max():.2f}, rho {ep[:, 1].min():.2f}..{ep[:, 1].max():.2f}, "
              f"{it_l} iterations, omega {om_l:.1f}")
    print(f"  paper          : overlaps {ov_p[1:]}, {it_p} iterations, omega {om_p:.1f}")
    it_l, ok_l, om_l, _ = out["level"]
    assert ok_p and ok_l and out["element"][1]
    # fewer iterations; omega (an operation-count model) is reported, the
    # benchmark judges the time to 1e-10
    assert it_l < it_p


def test_learned_per_element_cycle_matches_oracle(trained):
    """The network's per-element parameters on a small stretched problem: one
    V-cycle through the library equals the oracle's (Shepard-normalised
    per-element Schwarz, reading of the learned extension) to 1e-12."""
    from oracle.multigrid import Multigrid
    from paper_1512_02390_amd.sem import Solver
    learned, net, *_ = trained
    n, p = 6, 12
    xb = W.geometric_breaks(n, 1.0 / n, 16.0)
    yb = W.uniform_breaks(n, 1.0)
    NU = learned.nodal_nu(xb, yb, p, 0, W.GaussianFieldNu())
    base = Solver(xb, yb, p, 0, 1, 1, 5, nu=NU)
    ep = learned.predict(base, net)
    base.close()
    assert ep is not None
    ep = ep.astype(np.float32).astype(np.float64)
    s = Solver(xb, yb, p, 0, 1, 1, 5, nu=NU, elem_params=ep)
    mg = Multigrid(xb, yb, p, 0, 1, 1, 5, NU=NU,
                   elem_params=(ep[:, 0].reshape(n, n), ep[:, 1].reshape(n, n)))
    sp = mg.spaces[-1]
    U = W.random_guess(sp.shape, 0, 7)
    F = W.random_nodal(sp.shape, 0, 8)
    ns1, ns2 = [1] * (mg.L + 1), [1] * (mg.L + 1)
    ref = mg.vcycle(U, F, ns1, ns2)
    u = torch.tensor(U, dtype=torch.float64, device="cuda")
    s.vcycle(u, torch.tensor(F, dtype=torch.float64, device="cuda"), ns1, ns2)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    s.close()
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_unusable_prediction_falls_back_to_paper_parameters(trained):
    from paper_1512_02390_amd.sem import MLP
    learned = trained[0]
    bad = MLP(np.full(W.mlp_init().size, np.nan, dtype=np.float32))
    xb, yb, p = _problem()
    s, params = learned.solver_with_learned(xb, yb, p, 0, None, bad)
    assert params is None
    assert [s.level_info(l)[1] for l in range(1, s.L + 1)] == [1, 1, 1, 2]
    s.close()
    bad.close()
