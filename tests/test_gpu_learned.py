"""The learned Schwarz parameters end to end on the GPU: training data from
the solver's own sweeps, training with the library's kernels, and the gain of
the trained network over the paper's parameters (ceil(p_l/8) overlap, full
transition width) on a held-out variable-diffusion problem on a stretched
mesh, measured as the cost per decade of residual reduction
omega = W / r_bar of the full MGCG solve to 1e-10 (at most 300 iterations)."""
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
    n, p = 16, 12
    xb = W.geometric_breaks(n, 1.0 / n, 16.0)
    yb = W.uniform_breaks(n, 1.0)
    return xb, yb, p


def _solve(s, fn, kind="mg11"):
    from paper_1512_02390_amd import learned
    shape = s.shape()
    b = s.zeros()
    s.mass(torch.tensor(fn, dtype=torch.float64, device="cuda"), b)
    u = torch.tensor(W.random_guess(shape, 0, W.SEED_U0), dtype=torch.float64, device="cuda")
    ns1, ns2 = learned.schedule(s.L, kind)
    it, hist, ok = s.pcg_solve(u, b, 300, 1e-10, ns1, ns2)
    ov = [0] + [s.level_info(l)[1] for l in range(1, s.L + 1)]
    w = learned.cycle_cost(s.p, ov, [a + c for a, c in zip(ns1, ns2)])
    return it, ok, w / learned.rbar(hist), ov


def test_learned_parameters_beat_the_paper_on_held_out_problem(trained):
    from paper_1512_02390_amd.sem import SemError, Solver
    learned, net, *_ = trained
    xb, yb, p = _problem()
    NU = learned.nodal_nu(xb, yb, p, 0, W.GaussianFieldNu())
    fn = W.random_nodal(NU.shape, 0, W.SEED_RHS)
    paper = Solver(xb, yb, p, 0, 1, 1, 5, nu=NU)
    ov_p = [0] + [paper.level_info(l)[1] for l in range(1, paper.L + 1)]
    try:
        it_p, ok_p, om_p, ov_p = _solve(paper, fn)
    except SemError:
        # the paper's parameters stagnate on this problem; rounding can tip
        # the iteration into overflow: no reduction at all
        it_p, ok_p, om_p = 300, False, math.inf
    paper.close()
    s, params = learned.solver_with_learned(xb, yb, p, 0, NU, net)
    assert params is not None
    it_l, ok_l, om_l, ov_l = _solve(s, fn)
    s.close()
    print(f"  paper  : overlaps {ov_p[1:]}, {it_p} iterations, omega {om_p:.1f}")
    print(f"  learned: overlaps {ov_l[1:]}, alpha {params[1].min():.2f}..{params[1].max():.2f}, "
          f"{it_l} iterations, omega {om_l:.1f}")
    # the learned parameters must converge; the paper's may not (then its
    # omega comes from the residual reduction reached in 300 iterations)
    assert ok_l
    assert om_l < om_p


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
