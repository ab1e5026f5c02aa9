"""relax_diagnostics_noalloc (the entry point for callers that cannot allocate) against
relax_diagnostics of a context holding the same positions and field: E_M, xi, R2, min det F
and the concave-node count agree bit for bit (the same sweep kernels; the prescaling of B0
happens as it is loaded instead of in a copy, with the same rounding).  Three calls in a row
on one device, each on a smaller grid than the one before, so the second and third find the
previous call's contents in the shared scratch."""
import numpy as np
import pytest

import paper_1405_0942_amd as R
import workloads as W
from gpu_util import banner, context, dev, host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

FIELDS = ("E_M", "xi", "R2", "min_det", "concave")


def _concave_case(n, bc, amp, width):
    g = W.make_grid(n, [(-1.0, 1.3), (-0.4, 0.6), (-2.0, 2.0)], bc)
    x0 = W.distorted_grid(g, 0.05 * min(g.h), seed=5) + W.checkerboard_bump(g, amp, width)
    B0 = W.smooth_random_field(g, 0.6, seed=200) + np.array([0.2, -0.1, 1.0])[:, None, None, None]
    return g, x0, B0


def _compare(g, x, B0, steps=0, dt=1e-3, curl=R.RELAX_CURL_NN):
    cfg = R.make_config(g, dt0=dt, adaptive=False, curl=curl)
    with context(g, x, B0, dt0=dt, adaptive=False, curl=curl) as r:
        if steps:
            r.step(steps)
        ref = r.diagnostics()
        xs = r.state()[0]
        B0d = dev(B0)
        torch.cuda.synchronize()
        rc, d = R.relax_diagnostics_noalloc(cfg, xs.data_ptr(), B0d.data_ptr(), r.stream.cuda_stream)
        assert rc == R.RELAX_OK, R.relax_strerror(rc)
    got = {f: getattr(d, f) for f in FIELDS}
    banner(f"  {tuple(g.n)}: noalloc {got} | relax_diagnostics {[ref[f] for f in FIELDS]}")
    for f in FIELDS:
        assert got[f] == ref[f], (f, got[f], ref[f])
    assert d.t == 0.0 and d.dt == dt and d.Lambda == 0.0 and d.rejects == 0
    return got


def test_noalloc_diagnostics_match_context_three_calls_shrinking():
    banner("noalloc: abc 96^3 after 10 fixed steps")
    w = W.abc_box(96)
    got = _compare(w.grid, w.x0, w.B0, steps=10, dt=5e-4)
    assert got["xi"] > 0.0
    banner("noalloc: concave case 70 x 11 x 37, bc (1, 1, 0)")
    got = _compare(*_concave_case((70, 11, 37), (1, 1, 0), 0.8, 4.0))
    assert got["concave"] > 0
    banner("noalloc: concave case 20 x 18 x 16, line-tied")
    got = _compare(*_concave_case((20, 18, 16), (0, 0, 0), 0.7, 3.0))
    assert got["concave"] > 0


def test_noalloc_diagnostics_octilateral_current():
    """The same comparison with the octilateral current of Sec. 2.3, whose sweep the entry point
    runs when the configuration asks for it; xi differs from the nearest-neighbour value, so the
    octilateral sweep is the one that ran."""
    for n, bc in (((20, 18, 16), (0, 0, 0)), ((70, 11, 37), (1, 1, 0))):
        banner(f"noalloc, octilateral: concave case {n}, bc {bc}")
        case = _concave_case(n, bc, 0.3, 4.0)
        got = _compare(*case, curl=R.RELAX_CURL_NNN)
        nn = _compare(*case)
        assert got["E_M"] == nn["E_M"] and got["min_det"] == nn["min_det"]
        assert got["xi"] != nn["xi"] and got["R2"] != nn["R2"]
