"""Mixed precision (reduced-precision V-cycle inside FP64 residual and CG):
error against the FP64 oracle, stated per result and precision.

  - FP32 V-cycle: one cycle u <- u + MG32(0, f - A u) differs from the
    oracle's FP64 V-cycle by FP32 rounding only: relative error below 2e-5;
  - BF16 matrix-core subdomain solves (tiles of 17 nodes or more; FP32
    accumulation, the rest FP32): BF16 operand rounding (unit roundoff 2^-9)
    through four products, relative error below 3e-2 (about 15 unit
    roundoffs);
  - FP16 matrix-core subdomain solves (operand tiles scaled by powers of two):
    unit roundoff 2^-11, the same 15 unit roundoffs: below 8e-3;
  - mixed MGCG reaches a true FP64 residual of 1e-10 (recomputed by the
    oracle), in at most two (FP32) or four (BF16, FP16) iterations more than FP64,
    and its solution matches the oracle's FP64 solution (solved to 1e-13) to
    1e-8 relative.
"""
import sys

import numpy as np
import pytest

from parity_cases import CASES, P, build_gpu, build_oracle, rel_err
from paper_1512_02390_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MIXED, BF16, FP16 = 1, 2, 3
VCYCLE_TOL = {MIXED: 2e-5, BF16: 3e-2, FP16: 8e-3}
EXTRA_ITERS = {MIXED: 2, BF16: 4, FP16: 4}
NAME = {MIXED: "fp32", BF16: "bf16", FP16: "fp16"}
SUBSET = [c for c in CASES if c.name in ("dir_p4_no1", "dir_p8_no3_stretch", "per_p6_no2_cubic",
                                         "dir_p16_ceil8", "dir_p12_ceil8_varnu_stretch",
                                         "dir_p32_ceil8", "dir_p32_levels_varnu_stretch",
                                         "dir_p16_sep_strong",
                                         "dir_p12_elem_varnu_stretch", "dir_p32_elem")]


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module", params=[(c, pr) for pr in (MIXED, BF16, FP16) for c in SUBSET],
                ids=lambda cp: f"{cp[0].name}-{NAME[cp[1]]}")
def pair(request):
    case, prec = request.param
    print(f"[gpu-mixed] {case.name} precision {prec}", flush=True)
    mg, NU = build_oracle(case)
    gpu = build_gpu(case, NU, precision=prec)
    gpu.prec = prec
    yield case, mg, gpu
    gpu.close()


def test_mixed_vcycle_error(pair):
    case, mg, gpu = pair
    sp = mg.spaces[-1]
    U = W.random_guess(sp.shape, case.bc, 90)
    F = W.random_nodal(sp.shape, case.bc, 91)
    if case.bc == P:
        F = np.where(sp.mask, F - F[sp.mask].mean(), 0.0)
    ref = mg.vcycle(U, F)
    u = _dev(U)
    gpu.vcycle(u, _dev(F))
    err = rel_err(_host(u), ref)
    print(f"  mixed V-cycle rel. error vs FP64 oracle: {err:.2e}")
    assert err < VCYCLE_TOL[gpu.prec]


def test_mixed_pcg_reaches_fp64_accuracy(pair):
    case, mg, gpu = pair
    from oracle.mgcg import mgcg
    sp = mg.spaces[-1]
    U0 = W.random_guess(sp.shape, case.bc, 92)
    F = W.random_nodal(sp.shape, case.bc, 93)
    Uref, hist_ref, it_ref = mgcg(mg, U0, F, 100, 1e-13)
    _, _, it64 = mgcg(mg, U0, F, 100, 1e-10)
    u = _dev(U0)
    it, hist, ok = gpu.pcg_solve(u, _dev(F), 100, 1e-10)
    assert ok
    Ug = _host(u)
    Fp = F - (F[sp.mask].mean() if case.bc == P else 0.0)
    r0 = np.linalg.norm(mg.residual(mg.L, U0, sp.zero_boundary(Fp))[sp.mask])
    r = np.linalg.norm(mg.residual(mg.L, Ug, sp.zero_boundary(Fp))[sp.mask])
    if case.bc == P:
        Ug = Ug - Ug.mean()
        Uref = Uref - Uref.mean()
    err = rel_err(Ug, Uref)
    print(f"  mixed MGCG: {it} iterations (FP64 oracle {it64}), true residual ratio "
          f"{r / r0:.2e}, rel. error vs FP64 solution {err:.2e}")
    assert r <= 2e-10 * r0
    assert it <= it64 + EXTRA_ITERS[gpu.prec]
    assert err < 1e-8


@pytest.mark.parametrize("prec", [BF16, FP16], ids=["bf16", "fp16"])
def test_matrix_core_cycle_is_scale_invariant(prec):
    """The V-cycle is linear, so MG(0, 2^k f) = 2^k MG(0, f).  Powers of two
    are exact in every format used, so this holds up to the run-to-run order
    of the atomic scatter (FP32 level) -- provided no operand leaves its
    format's range.  For FP16 operands that takes the per-tile scaling: 2^-70
    would flush every FP16 operand to zero and 2^40 would overflow it."""
    case = next(c for c in CASES if c.name == "dir_p16_ceil8")
    mg, NU = build_oracle(case)
    gpu = build_gpu(case, NU, precision=prec)
    try:
        sp = mg.spaces[-1]
        F = W.random_nodal(sp.shape, case.bc, 94)
        u1 = gpu.zeros()
        gpu.vcycle(u1, _dev(F))
        ref = _host(u1)
        assert np.abs(ref).max() > 0
        for k in (-70, 40):
            uk = gpu.zeros()
            gpu.vcycle(uk, _dev(np.ldexp(F, k)))
            got = np.ldexp(_host(uk), -k)
            err = rel_err(got, ref)
            print(f"  {NAME[prec]} V-cycle of 2^{k} f, scaled back: rel. difference {err:.1e}")
            assert err < 1e-5
    finally:
        gpu.close()
