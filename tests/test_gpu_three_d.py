"""GPU parity of the 3-D extension (sem3_*) against the 3-D oracle on the same
seeded inputs, element by element, FP64 tolerance 1e-12 relative to the
largest entry: residual and operator, Schwarz sweeps, transfers, coarse
solve, V-cycles and the MGCG solve (iterations equal, history and solution
to 1e-12).  Cases: uniform and stretched meshes, fixed and ceil(p_l/8)
overlaps, n_o = 0, quintic, cubic and top-hat weights, a single element, and
a coarse grid too long for the one-workgroup coarse solve."""
from dataclasses import dataclass

import numpy as np
import pytest

from parity_cases import rel_err
from paper_1512_02390_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-12


@dataclass(frozen=True)
class Case3:
    name: str
    n: tuple           # elements along x, y, z
    p: int
    rule: int = 0      # 0 fixed, 1 ceil(p_l/8)
    n_o: int = 1
    wf: int = 5
    stretched: bool = False

    def breaks(self):
        nx, ny, nz = self.n
        if self.stretched:
            return (W.geometric_breaks(nx, 0.3, 2.5), W.uniform_breaks(ny, 0.8),
                    W.geometric_breaks(nz, 0.5, 1.6))
        return W.uniform_breaks(nx, 1.0), W.uniform_breaks(ny, 1.0), W.uniform_breaks(nz, 1.0)


CASES3 = [
    Case3("p4_no1", (3, 2, 2), 4),
    Case3("p6_no2_stretch_cubic", (2, 3, 2), 6, n_o=2, wf=3, stretched=True),
    Case3("p8_ceil8_stretch", (2, 2, 3), 8, rule=1, stretched=True),
    Case3("p5_no0_tophat", (2, 2, 2), 5, n_o=0, wf=-1),
    Case3("p7_single_element", (1, 1, 1), 7, n_o=3),
    # 20 elements along x: 19 coarse unknowns, beyond the one-workgroup coarse
    # solve (band products along each axis instead)
    Case3("p2_no1_long_x", (20, 2, 2), 2),
]


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rand(sp, seed, kind="nodal"):
    g = W.rng(seed)
    a = g.uniform(-1.0, 1.0, size=sp.shape) if kind == "nodal" else g.uniform(0.0, 1.0, size=sp.shape)
    return sp.zero_boundary(a)


@pytest.fixture(scope="module", params=CASES3, ids=lambda c: c.name)
def pair3(request):
    from oracle.three_d import Multigrid3
    from paper_1512_02390_amd.sem import Solver3
    c = request.param
    print(f"[gpu-3d] {c.name}", flush=True)
    xb, yb, zb = c.breaks()
    mg = Multigrid3(xb, yb, zb, c.p, c.rule, c.n_o, c.wf)
    gpu = Solver3(xb, yb, zb, c.p, c.rule, c.n_o, c.wf)
    yield c, mg, gpu
    gpu.close()


def test_levels(pair3):
    c, mg, gpu = pair3
    assert gpu.L == mg.L
    for l in range(mg.L + 1):
        p, no, shape = gpu.level_info(l)
        assert p == mg.orders[l] and shape == mg.spaces[l].shape
        if l > 0:
            assert no == mg.overlaps[l]


def test_residual_and_operator(pair3):
    c, mg, gpu = pair3
    for l in range(mg.L + 1):
        sp = mg.spaces[l]
        U, F = _rand(sp, 10 + l, "u"), _rand(sp, 20 + l)
        r = gpu.zeros(l)
        gpu.residual(l, _dev(U), _dev(F), r)
        assert rel_err(_host(r), mg.residual(l, U, F)) < TOL, l
        gpu.residual(l, _dev(U), None, r)
        assert rel_err(_host(r), mg.op(l, U)) < TOL, l


def test_schwarz_smooth(pair3):
    c, mg, gpu = pair3
    for l in range(1, mg.L + 1):
        sp = mg.spaces[l]
        U, F = _rand(sp, 30 + l, "u"), _rand(sp, 40 + l)
        u = _dev(U)
        gpu.schwarz_smooth(l, u, _dev(F), 2)
        assert rel_err(_host(u), mg.smooth(l, U, F, 2)) < TOL, l


def test_transfers(pair3):
    c, mg, gpu = pair3
    for l in range(1, mg.L + 1):
        sf, sc = mg.spaces[l], mg.spaces[l - 1]
        R = _rand(sf, 50 + l)
        fc = gpu.zeros(l - 1)
        gpu.restrict(l, _dev(R), fc)
        assert rel_err(_host(fc), mg.restrict(l, R)) < TOL, ("restrict", l)
        Uc, Uf = _rand(sc, 60 + l), _rand(sf, 70 + l)
        uf = _dev(Uf)
        gpu.prolong_add(l, _dev(Uc), uf)
        assert rel_err(_host(uf), Uf + mg.prolong(l, Uc)) < TOL, ("prolong", l)


def test_coarse_solve(pair3):
    c, mg, gpu = pair3
    F = _rand(mg.spaces[0], 80)
    u0 = gpu.zeros(0)
    gpu.coarse_solve(_dev(F), u0)
    ref = mg.coarse_solve(F)
    if np.abs(ref).max() == 0.0:          # no coarse unknowns (single element)
        assert np.abs(_host(u0)).max() == 0.0
    else:
        assert rel_err(_host(u0), ref) < TOL


def test_vcycle(pair3):
    c, mg, gpu = pair3
    sp = mg.spaces[-1]
    U, F = _rand(sp, 90, "u"), _rand(sp, 91)
    u, f = _dev(U), _dev(F)
    for k in range(3):
        U = mg.vcycle(U, F)
        gpu.vcycle(u, f)
        assert rel_err(_host(u), U) < TOL, k


def test_pcg(pair3):
    from oracle.mgcg import mgcg
    c, mg, gpu = pair3
    sp = mg.spaces[-1]
    U0, F = _rand(sp, 92, "u"), _rand(sp, 93)
    Uref, hist_ref, it_ref = mgcg(mg, U0, F, 60, 1e-10)
    u = _dev(U0)
    it, hist, ok = gpu.pcg_solve(u, _dev(F), 60, 1e-10)
    assert ok and it == it_ref
    assert np.abs(hist - hist_ref).max() <= TOL * hist_ref[0]
    assert rel_err(_host(u), Uref) < TOL
