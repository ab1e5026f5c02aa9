"""IsoHelix accuracy runs (Sec. 3.1, 3.2; the mimetic rows of Table 1; FP64 and FP32-mixed).

The IsoHelix field (eq. "B init analytical": B0 = 1, a_r = sqrt 2, a_z = 2) of twist angle
phi = pi/4, pi/2 or pi on odd vertex grids n^3 over [-4, 4]^2 x [-10, 10], all faces
line-tied, x0 = X, relaxed with the adaptive step (Lambda0 = 1e-8, safety 0.9, dt_min 1e-9)
until sigma_B and sigma_x settle (1e-3 over two chunks); B and J of the relaxed state come
from relax_fields (checked against the oracle's fields of the same positions).

sigma_B, sigma_x and eps* (definitions in isohelix_util) are compared with the values the
paper prints in Table 1 (tests/golden/isohelix_table1_mimetic.txt) within 30 %, and must
fall with resolution as the paper reports for phi = pi/4.  Where the paper marks a run as not
converging (phi = pi, n = 17) the run must end in the step-size collapse.  The paper ran the
pi/2 and pi rows in single precision; these runs are FP64, and the pi/4 and pi/2 rows at
n = 17, 33 also in the FP32-mixed mode.  xi is not compared: it keeps falling with the run
length and depends on Lambda0 (the paper says so, Sec. 4.1), neither of which the paper
states; it must only show that the field relaxed.  RELAX_ISOHELIX_FULL=1 adds n = 129 for
phi = pi/4.  At n = 129 the pi/2 and pi runs (FP64 and FP32-mixed alike) reach smaller
eps* and sigma_B than the paper's single-precision rows print (by up to 3x).  The cause of
that deviation is not known (one hypothesis: the single precision of those runs of the paper,
or run lengths it does not give), so those rows are reported in the design notes and not
compared.
"""
import os

import numpy as np
import pytest

import oracle
import paper_1405_0942_amd as R
import workloads as W
from gpu_util import banner, context, host, nrel
from isohelix_util import PHIS, grid, relaxed_state_errors, table1

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

FULL = os.environ.get("RELAX_ISOHELIX_FULL") == "1"
SIZES = (17, 33, 65)


def relax(n, phi, max_steps=200_000, precision=R.RELAX_FP64):
    """(grid, B0, x, B, J, final diagnostics, steps, status) of a run to the relaxed state."""
    g = grid(n)
    B0 = W.isohelix_field(g, phi)
    with context(g, g.identity(), B0, dt0=1e-3, tol=1e-8, safety=0.9, dt_min=1e-9, precision=precision) as r:
        done, chunk, hist = 0, 250, []
        while done < max_steps:
            d = r.step(chunk, raise_on_error=False)
            done += len(d)
            if r.last_status != R.RELAX_OK:
                banner(f"  n {n}: status {r.last_status} after {done} steps")
                return g, B0, None, None, None, None, done, r.last_status
            x = host(r.state()[0])
            Bt, Jt = r.fields()
            B, J = host(Bt), host(Jt)
            sB, sx, eps = relaxed_state_errors(g, x, B, J, phi)
            hist.append((sB, sx))
            banner(f"  n {n}: step {done}, t {d[-1]['t']:.1f}, dt {d[-1]['dt']:.3e}, xi {d[-1]['xi']:.2e}, "
                   f"sigma_B {sB:.3e}, sigma_x {sx:.3e}, eps* {eps:.2e}")
            if len(hist) >= 3 and all(abs(hist[-1][k] - hist[-3][k]) <= 1e-3 * hist[-1][k] for k in (0, 1)):
                break
            chunk = min(2 * chunk, 16_000)
        fin = r.diagnostics()
    return g, B0, x, B, J, fin, done, R.RELAX_OK


# n = 129 (RELAX_ISOHELIX_FULL=1) only for the double-precision pi/4 row: the paper's single-
# precision pi/2 and pi rows at n = 129 lie above what these runs reach (see the module text)
CASES = [("pi/4", "fp64", SIZES + ((129,) if FULL else ())), ("pi/2", "fp64", SIZES), ("pi", "fp64", SIZES),
         ("pi/4", "mixed", (17, 33)), ("pi/2", "mixed", (17, 33))]


@pytest.mark.parametrize("phi,prec,sizes", CASES, ids=[f"{c[0]}-{c[1]}" for c in CASES])
def test_isohelix_relaxed_state_matches_table1(phi, prec, sizes):
    """FP32-mixed runs (FP32 stencil, FP64 positions and control) reach the same relaxed
    states: the asymptotic errors are set by the discretisation, not the arithmetic."""
    paper = table1(phi)
    table = {}
    for n in sizes:
        banner(f"IsoHelix phi = {phi}, {n}^3, {prec}")
        g, B0, x, B, J, fin, steps, status = relax(
            n, PHIS[phi], precision=R.RELAX_FP64 if prec == "fp64" else R.RELAX_FP32_MIXED)
        p = paper[n]
        if p is None:  # the paper's run did not converge
            assert status == R.RELAX_E_DT, status
            banner(f"n {n}: breaks down after {steps} steps | Table 1: no converged values")
            continue
        assert status == R.RELAX_OK
        sB, sx, eps = relaxed_state_errors(g, x, B, J, PHIS[phi])
        table[n] = (fin["xi"], eps, sB, sx)
        o = oracle.fields(g, x, B0)
        assert nrel(B, o["B"]) < 1e-12 and nrel(J, o["J"]) < 1e-11
        banner(f"n {n}: xi {fin['xi']:.2e} eps* {eps:.2e} sigma_B {sB:.2e} sigma_x {sx:.2e} ({steps} steps) | "
               f"Table 1: eps* {p[1]:.1e} sigma_B {p[2]:.1e} sigma_x {p[3]:.1e}")
        for k in (1, 2, 3):
            assert 1 / 1.3 < table[n][k] / p[k] < 1.3, (n, k, table[n][k], p[k])
        assert fin["xi"] < 1e-4
    ns = sorted(table)
    for a, b in zip(ns, ns[1:]):
        assert table[b][2] < 0.5 * table[a][2]  # sigma_B falls with resolution
        assert table[b][1] < table[a][1]  # eps* falls with resolution
        if phi == "pi/4":
            assert table[b][3] <= 1.05 * table[a][3]  # sigma_x does not grow
