"""GPU parity: every entry point of the C-ABI against the oracle on the same
seeded inputs, element by element, FP64 tolerance 1e-12 relative to the
largest entry (operators with atomic accumulation differ from the oracle
only by rounding order).  The same bound holds for the coarse solve, three
V-cycles and the whole MGCG solve (residual history relative to ||r_0||, final
iterate relative to its largest entry): measured differences are at most
1e-13 on every case."""
import sys

import numpy as np
import pytest

from parity_cases import CASES, P, build_gpu, build_oracle, rel_err
from paper_1512_02390_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _announce(name):
    print(f"[gpu-parity] {name}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=CASES, ids=lambda c: c.name)
def pair(request):
    case = request.param
    _announce(case.name)
    mg, NU = build_oracle(case)
    gpu = build_gpu(case, NU)
    yield case, mg, gpu
    gpu.close()


def test_layout_and_coordinates(pair):
    case, mg, gpu = pair
    assert gpu.nlevels == mg.L + 1
    for l in range(mg.L + 1):
        pl, no, r, c = gpu.level_info(l)
        assert pl == mg.orders[l]
        assert (r, c) == mg.spaces[l].shape
        if l > 0:
            assert no == mg.overlaps[l]
        x, y = gpu.node_coords(l)
        assert np.allclose(x, mg.spaces[l].x(), atol=1e-14)
        assert np.allclose(y, mg.spaces[l].y(), atol=1e-14)


def test_residual(pair):
    case, mg, gpu = pair
    for l in range(mg.L + 1):
        sp = mg.spaces[l]
        U = W.random_guess(sp.shape, case.bc, 10 + l)
        F = W.random_nodal(sp.shape, case.bc, 20 + l)
        ref = mg.residual(l, U, F)
        r = gpu.zeros(l)
        gpu.residual(l, _dev(U), _dev(F), r)
        assert rel_err(_host(r), ref) < TOL, (l,)
        # f = NULL gives A u
        gpu.residual(l, _dev(U), None, r)
        assert rel_err(_host(r), mg.op(l, U)) < TOL


def test_schwarz_smooth(pair):
    case, mg, gpu = pair
    for l in range(1, mg.L + 1):
        sp = mg.spaces[l]
        U = W.random_guess(sp.shape, case.bc, 30 + l)
        F = W.random_nodal(sp.shape, case.bc, 40 + l)
        ref = mg.smooth(l, U, F, 2)
        u = _dev(U)
        gpu.schwarz_smooth(l, u, _dev(F), 2)
        assert rel_err(_host(u), ref) < TOL, (l,)


def test_transfers(pair):
    case, mg, gpu = pair
    for l in range(1, mg.L + 1):
        sf, sc = mg.spaces[l], mg.spaces[l - 1]
        R = W.random_nodal(sf.shape, case.bc, 50 + l)
        fc = gpu.zeros(l - 1)
        gpu.restrict(l, _dev(R), fc)
        assert rel_err(_host(fc), mg.restrict(l, R)) < TOL, ("restrict", l)
        Uc = W.random_nodal(sc.shape, case.bc, 60 + l)
        Uf = W.random_nodal(sf.shape, case.bc, 70 + l)
        uf = _dev(Uf)
        gpu.prolong_add(l, _dev(Uc), uf)
        assert rel_err(_host(uf), Uf + mg.prolong(l, Uc)) < TOL, ("prolong", l)


def test_coarse_solve(pair):
    case, mg, gpu = pair
    s0 = mg.spaces[0]
    F = W.random_nodal(s0.shape, case.bc, 80)
    u0 = gpu.zeros(0)
    gpu.coarse_solve(_dev(F), u0)
    assert rel_err(_host(u0), mg.coarse_solve(F)) < TOL


def test_vcycle(pair):
    case, mg, gpu = pair
    sp = mg.spaces[-1]
    U = W.random_guess(sp.shape, case.bc, 90)
    F = W.random_nodal(sp.shape, case.bc, 91)
    if case.bc == P:
        F = np.where(sp.mask, F - F[sp.mask].mean(), 0.0)
    u = _dev(U)
    f = _dev(F)
    ns1 = [1] * (mg.L + 1)
    ns2 = [1 if case.varnu else 0] * (mg.L + 1)
    for k in range(3):
        U = mg.vcycle(U, F, ns1, ns2)
        gpu.vcycle(u, f, ns1, ns2)
        err = rel_err(_host(u), U)
        assert err < TOL, (k, err)


def test_pcg(pair):
    case, mg, gpu = pair
    from oracle.mgcg import mgcg
    sp = mg.spaces[-1]
    U0 = W.random_guess(sp.shape, case.bc, 92)
    F = W.random_nodal(sp.shape, case.bc, 93)
    Uref, hist_ref, it_ref = mgcg(mg, U0, F, 60, 1e-10)
    u = _dev(U0)
    it, hist, ok = gpu.pcg_solve(u, _dev(F), 60, 1e-10)
    assert ok and it == it_ref
    assert np.abs(hist - hist_ref).max() <= TOL * hist_ref[0]
    Ug = _host(u)
    if case.bc == P:
        Ug = Ug - Ug.mean()
        Uref = Uref - Uref.mean()
    assert rel_err(Ug, Uref) < TOL


def test_pcg_degenerate_cases():
    """Zero initial residual: no iteration, u unchanged (the algorithm's
    alpha would be 0/0).  imax = 0: not converged, u unchanged, the history
    holds the oracle's ||r_0||."""
    case = next(c for c in CASES if c.name == "dir_p4_no1")
    mg, NU = build_oracle(case)
    gpu = build_gpu(case, NU)
    try:
        sp = mg.spaces[-1]
        zero = np.zeros(sp.shape)
        u = _dev(zero)
        it, hist, ok = gpu.pcg_solve(u, _dev(zero), 20, 1e-10)
        assert ok and it == 0 and hist[0] == 0.0
        assert np.all(_host(u) == 0.0)
        U0 = W.random_guess(sp.shape, case.bc, 95)
        F = W.random_nodal(sp.shape, case.bc, 96)
        u = _dev(U0)
        it, hist, ok = gpu.pcg_solve(u, _dev(F), 0, 1e-10)
        assert not ok and it == 0
        r0 = np.linalg.norm(mg.residual(mg.L, U0, F)[sp.mask])
        assert abs(hist[0] - r0) <= 1e-12 * r0
        assert np.array_equal(_host(u), np.where(sp.mask, U0, 0.0)) or np.array_equal(_host(u), U0)
    finally:
        gpu.close()
