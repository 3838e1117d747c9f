"""GPU parity of the learned-parameter kernels against the FP64 oracle
(oracle/mlp.py): element features, the MLP forward pass, its gradient and
Adam steps, all through the C-ABI.  FP32 on the device, so tolerances follow
FP32 rounding: features and outputs to ~1e-6 absolute, gradients to 1e-4
relative (2-norm), Adam trajectories to 1 % of the distance travelled."""
import numpy as np
import pytest

from oracle import mlp
from parity_cases import CASES, build_oracle, nu_field
from paper_1512_02390_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FEATURE_CASES = [c for c in CASES if c.name in ("dir_p4_no1", "dir_p8_no3_stretch",
                                                 "per_p6_no2_cubic", "dir_p12_ceil8_varnu_stretch",
                                                 "per_p8_varnu", "dir_p32_levels_varnu_stretch",
                                                 "dir_single_element_p9", "dir_p1")]


def _f32(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("case", FEATURE_CASES, ids=lambda c: c.name)
def test_features_match_oracle(case):
    from paper_1512_02390_amd.sem import Solver
    print(f"[gpu-mlp] features {case.name}", flush=True)
    mg, NU = build_oracle(case)
    xb, yb = case.breaks()
    s = Solver(xb, yb, case.p, case.bc, case.rule, case.n_o, case.wf, nu=NU)
    got = s.elem_features().cpu().numpy()
    s.close()
    ref = mlp.element_features(xb, yb, case.p, case.bc, NU)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 2e-6 * max(1.0, np.abs(ref).max())


def _theta(seed=7):
    return (W.mlp_init() + 0.05 * W.rng(seed).normal(size=mlp.n_params())).astype(np.float32)


def _batch(n, seed=8):
    g = W.rng(seed)
    X = g.normal(size=(n, 8)).astype(np.float32)
    T = g.uniform(0.05, 0.95, size=(n, 2)).astype(np.float32)
    return X, T


@pytest.mark.parametrize("n", [1, 37, 1000])
def test_forward_matches_oracle(n):
    from paper_1512_02390_amd.sem import MLP
    print(f"[gpu-mlp] forward n={n}", flush=True)
    th = _theta()
    X, _ = _batch(n)
    net = MLP(th)
    y = net.forward(_f32(X)).cpu().numpy()
    ref, _ = mlp.forward(th.astype(np.float64), X.astype(np.float64))
    assert np.abs(y - ref).max() <= 2e-6
    assert np.array_equal(net.get_params(), th)
    net.close()


@pytest.mark.parametrize("n", [1, 37, 1000])
def test_gradient_matches_oracle(n):
    from paper_1512_02390_amd.sem import MLP
    print(f"[gpu-mlp] gradient n={n}", flush=True)
    th = _theta()
    X, T = _batch(n)
    net = MLP(th)
    loss, g = net.gradient(_f32(X), _f32(T))
    g = g.cpu().numpy().astype(np.float64)
    L_ref, g_ref = mlp.gradient(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert loss == pytest.approx(L_ref, rel=1e-5)
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    for a, b in zip(mlp.unpack(g), mlp.unpack(g_ref)):     # every block, not just the largest
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-9
    # deterministic: the same call gives the same bits
    loss2, g2 = net.gradient(_f32(X), _f32(T))
    assert loss2 == loss and np.array_equal(g2.cpu().numpy().astype(np.float64), g)
    net.close()


def test_adam_steps_follow_oracle():
    from paper_1512_02390_amd.sem import MLP
    print("[gpu-mlp] adam", flush=True)
    th = _theta()
    X, T = _batch(200)
    net = MLP(th)
    opt = mlp.Adam(th.astype(np.float64))
    lr = 2e-3
    Xd, Td = _f32(X), _f32(T)
    for k in range(10):
        l_gpu = net.train_step(Xd, Td, lr, want_loss=True)
        l_ref, g_ref = mlp.gradient(opt.theta, X.astype(np.float64), T.astype(np.float64))
        opt.step(g_ref, lr)
        assert l_gpu == pytest.approx(l_ref, rel=1e-4)
    got = net.get_params().astype(np.float64)
    travelled = np.linalg.norm(opt.theta - th)
    assert travelled > 0
    assert np.linalg.norm(got - opt.theta) <= 0.01 * travelled
    net.close()


def test_training_on_device_fits_a_smooth_target():
    from paper_1512_02390_amd.sem import MLP
    print("[gpu-mlp] training", flush=True)
    g = W.rng(12)
    X = g.normal(size=(512, 8)).astype(np.float32)
    T = np.stack([1 / (1 + np.exp(-X[:, 0])), 0.5 + 0.4 * np.tanh(X[:, 1] * X[:, 2])],
                 1).astype(np.float32)
    net = MLP(W.mlp_init())
    Xd, Td = _f32(X), _f32(T)
    l0 = net.train_step(Xd, Td, 3e-3, want_loss=True)
    for _ in range(600):
        net.train_step(Xd, Td, 3e-3)
    l1 = net.train_step(Xd, Td, 3e-3, want_loss=True)
    print(f"  loss {l0:.3e} -> {l1:.3e}")
    assert l1 < 0.05 * l0
    net.close()
