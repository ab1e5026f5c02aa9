"""Per-node results do not depend on the workgroup tile: the library built with 64 x 4 tiles
(tests only) against the 64 x 8 build, bit for bit.  A different tile height changes the LDS
windows, the halo rings each thread loads, the own-node carry of the stage sweeps and the
z-chunking, but not the arithmetic of any node, so an LDS race or a halo mistake would show as
a difference.  Positions after a few steps (adaptive: the step-size rule reads only the max of
the error estimate, which does not depend on the order of the reduction), u, B and J, alpha*
and the convexity map are compared exactly; the energy sums only to rounding."""
import numpy as np
import pytest

import paper_1405_0942_amd as R
from paper_1405_0942_amd import build as B
import workloads as W
from gpu_util import banner, context, host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


def _concave_case(n, bc, amp, width):
    g = W.make_grid(n, [(-1.0, 1.3), (-0.4, 0.6), (-2.0, 2.0)], bc)
    x0 = W.distorted_grid(g, 0.05 * min(g.h), seed=5) + W.checkerboard_bump(g, amp, width)
    B0 = W.smooth_random_field(g, 0.6, seed=200) + np.array([0.2, -0.1, 1.0])[:, None, None, None]
    return g, x0, B0


CASES = {
    "abc_96_fp64_adaptive": (lambda: (W.abc_box(96).grid, W.abc_box(96).x0, W.abc_box(96).B0),
                             dict(dt0=5e-4, adaptive=True, tol=1e-7), 6),
    "abc_96_mixed_adaptive": (lambda: (W.abc_box(96).grid, W.abc_box(96).x0, W.abc_box(96).B0),
                              dict(dt0=5e-4, adaptive=True, tol=1e-7, precision=R.RELAX_FP32_MIXED), 6),
    "concave_70x11x37_pxy": (lambda: _concave_case((70, 11, 37), (1, 1, 0), 0.8, 4.0),
                             dict(dt0=1e-3, adaptive=False), 4),
    "concave_20x18x16_lt": (lambda: _concave_case((20, 18, 16), (0, 0, 0), 0.7, 3.0),
                            dict(dt0=1e-3, adaptive=False), 4),
    "twist_16_lt_adaptive": (lambda: (W.single_twist_16().grid, W.single_twist_16().x0, W.single_twist_16().B0),
                             dict(dt0=2e-3, adaptive=True, tol=1e-8), 5),
}


def _run(g, x0, B0, kw, steps):
    with context(g, x0, B0, **kw) as r:
        diag = r.step(steps)
        x = host(r.state()[0])
        u = host(r.velocity())
        Bf, J = (host(t) for t in r.fields())
        alpha, kappa = (host(t) for t in r.monitors())
        fin = r.diagnostics()
    return diag, x, u, Bf, J, alpha, kappa, fin


@pytest.mark.parametrize("name", list(CASES))
def test_results_independent_of_tile_height(name):
    make, kw, steps = CASES[name]
    g, x0, B0 = make()
    banner(f"tiling {name}: 64 x 8")
    a = _run(g, x0, B0, kw, steps)
    banner(f"tiling {name}: 64 x 4")
    with R.using_library(B.LIB_TY4):
        b = _run(g, x0, B0, kw, steps)
    da, db = a[0], b[0]
    assert [d["dt"] for d in da] == [d["dt"] for d in db]
    assert [d["rejects"] for d in da] == [d["rejects"] for d in db]
    for what, va, vb in zip(("x", "u", "B", "J", "alpha", "kappa"), a[1:7], b[1:7]):
        assert np.array_equal(va, vb), (name, what, float(np.abs(va - vb).max()))
    assert a[7]["min_det"] == b[7]["min_det"] and a[7]["concave"] == b[7]["concave"]
    assert a[7]["xi"] == b[7]["xi"]
    assert rel(a[7]["E_M"], b[7]["E_M"]) < 1e-13 and rel(a[7]["R2"], b[7]["R2"]) < 1e-12
