"""Host-side parts of the learned-parameter extension against the oracle: the
library's reduction of predictions to setup parameters (sem_learned_params,
host code, no device needed) and the cost measure used to label the sweeps."""
import numpy as np
import pytest

from oracle import mlp
from paper_1512_02390_amd import workloads as W


def _lib():
    from paper_1512_02390_amd import sem
    try:
        sem.load_library()
    except OSError:
        pytest.skip("libsem.so not built")
    return sem


@pytest.mark.parametrize("nx,ny,p,bc", [(2, 1, 8, 0), (5, 3, 12, 0), (4, 6, 32, 0),
                                        (3, 4, 5, 1), (7, 7, 16, 1), (1, 1, 1, 0)])
def test_learned_params_match_oracle(nx, ny, p, bc):
    sem = _lib()
    g = W.rng(40 + nx * ny + p)
    pred = g.uniform(-0.2, 1.2, size=(nx * ny, 2)).astype(np.float32)
    ov, ax, ay = sem.learned_params(pred, nx, ny, p, bc)
    ov_o, ax_o, ay_o = mlp.setup_from_predictions(pred.astype(np.float64), nx, ny, p, bc)
    assert ov == ov_o
    assert np.allclose(ax, ax_o, rtol=1e-15, atol=0)
    assert np.allclose(ay, ay_o, rtol=1e-15, atol=0)


def test_learned_params_hand_example_and_errors():
    sem = _lib()
    ov, ax, ay = sem.learned_params(np.array([[0.5, 0.5], [1.0, 1.0]]), 2, 1, 8, 0)
    assert ov == [0, 1, 2, 3]
    assert np.allclose(ax, [0.5, 0.75, 1.0]) and np.allclose(ay, [0.75, 0.75])
    with pytest.raises(sem.SemError):
        sem.learned_params(np.array([[np.nan, 0.5]]), 1, 1, 4, 0)


def test_overlap_ratio_and_cost_match_oracle():
    _lib()
    from paper_1512_02390_amd import learned
    for p in (2, 4, 8, 12, 16, 32):
        for rho in learned.RATIOS:
            ov = learned.overlaps_for(rho, p)
            assert ov == mlp.overlaps_from_ratio(rho, p)
            L = len(ov) - 1
            for ns in ([2] * (L + 1), [2 ** (L - l + 1) for l in range(L + 1)]):
                assert learned.cycle_cost(p, ov, ns) == pytest.approx(mlp.cycle_cost(p, ov, ns),
                                                                      rel=1e-14)


def test_label_is_smallest_omega():
    from paper_1512_02390_amd import learned
    rows = [(1.0, 0.125, 1.0, 9.0), (0.5, 0.25, 1.5, 7.5), (0.25, 0.5, 0.0, float("inf"))]
    assert learned.label_of(rows) == (0.5, 0.5)
