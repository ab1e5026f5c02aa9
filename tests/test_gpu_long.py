"""Long runs of the braid workloads: FP64 against the oracle (64x64x192), and FP32-mixed
against FP64 (128x128x384).

* Braid 64x64x192, FP64, adaptive: the oracle replays the GPU's accepted dt sequence for
  the first 1000 steps (E_M, xi and the displacement compared step by step); the GPU then
  runs on to 4000 steps, and the oracle's diagnostics of the GPU's final positions must
  match the GPU's own FP64 diagnostics sweep of them.  (Run on, this discretization of the
  braid develops a grid-scale instability: xi bottoms out near 1.9e-2 around step 4250,
  then grows while E_M turns upward and det F collapses, and the step size falls below
  1e-12 at step 5440, t = 35.5.  The oracle replaying the GPU's whole dt sequence from x0
  follows the same path: test_braid_64_fp64_breakdown_replayed_from_x0, opt-in with
  RELAX_BRAID_BREAKDOWN=1.)
* Braid 128x128x384, FP64 and FP32-mixed, 5000 steps at the same fixed dt: E_M of every
  step and the final FP64-evaluated xi and R2 of the mixed run within 1e-5 relative of the
  FP64 run (the mixed mode keeps positions in FP64 and evaluates the final diagnostics with
  the FP64 sweep), and the final displacement x - X normwise within 1e-6 of the FP64 run's;
  the first 100 mixed steps also against the oracle (E_M of every step within 1e-5, the
  displacement after them within 1e-5).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import banner, context, host, nrel, rel

import paper_1405_0942_amd as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


def test_braid_64_fp64_long_run_vs_oracle():
    w = W.braid(64, 192)
    g = w.grid
    tau_B2 = oracle.null_threshold(w.B0)
    K_cmp, K_total = 1000, 4000
    banner(f"braid 64x64x192 FP64 adaptive: {K_cmp} steps vs oracle replay, then to {K_total}")
    with context(g, w.x0, w.B0, dt0=w.dt0, tol=w.tol) as r:
        diag = r.step(K_cmp)
        x_cmp = host(r.state()[0])
        rest = r.step(K_total - K_cmp)
        xK = host(r.state()[0])
        dK = r.diagnostics()
    gdt = np.array([d["dt"] for d in diag])
    ref = oracle.run(g, w.x0, w.B0, K_cmp, dt=gdt[0], mode=oracle.MODE_REPLAY, dts=gdt, tau_B2=tau_B2)
    od = ref["diag"]
    E = np.array([d["E_M"] for d in diag])
    xi = np.array([d["xi"] for d in diag])
    errE = np.abs(E - od[:, 2]).max() / E[0]
    errxi = np.abs(xi - od[:, 3]).max() / np.abs(od[:, 3]).max()
    errx = nrel(x_cmp - w.x0, ref["x"] - w.x0)
    banner(f"  {K_cmp} steps: E_M {errE:.2e}, xi {errxi:.2e}, displacement {errx:.2e}; "
           f"rejects {sum(d['rejects'] for d in diag)}")
    assert errE < 1e-11
    assert errxi < 1e-9
    assert errx < 1e-9
    # the rest of the run: energy decreases, and the final diagnostics agree with the oracle's
    # evaluation of the GPU's final positions
    E_all = np.concatenate([E, [d["E_M"] for d in rest]])
    assert np.all(E_all[1:] <= E_all[:-1] * (1 + 1e-13))
    assert dK["xi"] < 0.25 * diag[0]["xi"]
    o = oracle.diagnostics(g, xK, w.B0, tau_B2=tau_B2)
    banner(f"  step {K_total}: t {rest[-1]['t']:.4f}, E_M {dK['E_M']:.10g}, xi {dK['xi']:.3e}, "
           f"R2 {dK['R2']:.3e}; oracle diagnostics rel E {rel(dK['E_M'], o['E_M']):.1e} "
           f"xi {rel(dK['xi'], o['xi']):.1e} R2 {rel(dK['R2'], o['R2']):.1e}")
    assert rel(dK["E_M"], o["E_M"]) < 1e-12
    assert rel(dK["R2"], o["R2"]) < 1e-11
    assert rel(dK["xi"], o["xi"]) < 1e-11
    assert rel(dK["min_det"], o["min_det"]) < 1e-12


def _probe_dt(w, steps=40):
    """Smallest dt the adaptive FP64 run accepts over its first steps (a fixed dt below the
    stability limit of the whole run, whose steps only grow as the field relaxes)."""
    with context(w.grid, w.x0, w.B0, dt0=w.dt0, tol=w.tol) as r:
        d = r.step(steps)
    return min(x["dt"] for x in d)


def test_braid_128_mixed_vs_fp64():
    w = W.braid(128, 384)
    g = w.grid
    K = 5000
    dt = _probe_dt(w)
    banner(f"braid 128x128x384: FP64 and FP32-mixed, {K} steps at dt {dt:.4e}")
    runs = {}
    for prec in (R.RELAX_FP64, R.RELAX_FP32_MIXED):
        with context(g, w.x0, w.B0, dt0=dt, adaptive=False, precision=prec) as r:
            diag = r.step(K)
            fin = r.diagnostics()
            x = host(r.state()[0])
        runs[prec] = (np.array([d["E_M"] for d in diag]), fin, x, diag)
    E64, f64, x64, d64 = runs[R.RELAX_FP64]
    E32, f32, x32, d32 = runs[R.RELAX_FP32_MIXED]
    errE = float(np.max(np.abs(E32 - E64) / np.abs(E64)))
    banner(f"  E_M(t) max rel {errE:.2e}; final (FP64 sweep) E_M {rel(f32['E_M'], f64['E_M']):.2e} "
           f"xi {rel(f32['xi'], f64['xi']):.2e} ({f64['xi']:.3e} vs {f32['xi']:.3e}) "
           f"R2 {rel(f32['R2'], f64['R2']):.2e}; displacement {nrel(x32 - w.x0, x64 - w.x0):.2e}; "
           f"in-loop xi FP64 {d64[-1]['xi']:.3e} mixed {d32[-1]['xi']:.3e}")
    assert errE < 1e-5
    # FP32 stage vectors carry ~1e-6 relative error per evaluation; over the run the
    # displacement of the mixed run stays within 1e-6 of the FP64 run's (measured 5e-8)
    assert nrel(x32 - w.x0, x64 - w.x0) < 1e-6
    assert rel(f32["E_M"], f64["E_M"]) < 1e-5
    assert rel(f32["xi"], f64["xi"]) < 1e-5
    assert rel(f32["R2"], f64["R2"]) < 1e-5
    # the FP64 sweep of the mixed run's final positions is the oracle's diagnostics of them
    tau_B2 = oracle.null_threshold(w.B0)
    o = oracle.diagnostics(g, x32, w.B0, tau_B2=tau_B2)
    assert rel(f32["E_M"], o["E_M"]) < 1e-12
    assert rel(f32["R2"], o["R2"]) < 1e-11
    assert rel(f32["xi"], o["xi"]) < 1e-11
    # the first mixed steps against the oracle (a second mixed run, stopped after K_o steps)
    K_o = 100
    ref = oracle.run(g, w.x0, w.B0, K_o, dt=dt, mode=oracle.MODE_FIXED, tau_B2=tau_B2)
    with context(g, w.x0, w.B0, dt0=dt, adaptive=False, precision=R.RELAX_FP32_MIXED) as r:
        r.step(K_o, diag=False)
        x_o = host(r.state()[0])
    errEo = float(np.max(np.abs(E32[:K_o] - ref["diag"][:, 2]) / ref["diag"][:, 2]))
    errxo = nrel(x_o - w.x0, ref["x"] - w.x0)
    banner(f"  first {K_o} mixed steps vs oracle: E_M max rel {errEo:.2e}, displacement {errxo:.2e}")
    assert errEo < 1e-5
    assert errxo < 1e-5


@pytest.mark.skipif(__import__("os").environ.get("RELAX_BRAID_BREAKDOWN") != "1",
                    reason="about 7 minutes of oracle time: RELAX_BRAID_BREAKDOWN=1")
def test_braid_64_fp64_breakdown_replayed_from_x0():
    """The braid's late grid-scale instability belongs to the discretisation: the GPU runs the
    64x64x192 braid (FP64, adaptive) until the step size falls below dt_min, and the oracle
    replays the GPU's whole accepted dt sequence from x0 (in chunks, printing as it goes).  Up
    to the minimum of E_M, E_M of every step agrees within 1e-9; from there on both runs see E_M
    turn upward (which the continuum forbids) and min det F collapse by five orders of
    magnitude.  An instability amplifies every difference, so after the onset the two runs
    agree in kind, not to rounding: the minimum falls on the same step, and the final min det F
    of the two (near 1e-5) within 5 %."""
    w = W.braid(64, 192)
    g = w.grid
    tau_B2 = oracle.null_threshold(w.B0)
    banner("braid 64x64x192 FP64 adaptive: run to the breakdown")
    diag = []
    with context(g, w.x0, w.B0, dt0=w.dt0, tol=w.tol, dt_min=1e-12) as r:
        while len(diag) < 20000:
            d = r.step(500, raise_on_error=False)
            diag += d
            banner(f"  GPU step {len(diag)}: t {diag[-1]['t']:.3f}, dt {diag[-1]['dt']:.2e}, "
                   f"E_M {diag[-1]['E_M']:.10g}, xi {diag[-1]['xi']:.2e}, min det {diag[-1]['min_det']:.2e}")
            if r.last_status != R.RELAX_OK:
                break
        status = r.last_status
    assert status == R.RELAX_E_DT
    gdt = np.array([d["dt"] for d in diag])
    E = np.array([d["E_M"] for d in diag])
    x, t = w.x0.copy(), 0.0
    oE, omin = [], []
    for s0 in range(0, len(gdt), 500):
        seg = gdt[s0:s0 + 500]
        o = oracle.run(g, x, w.B0, len(seg), dt=seg[0], mode=oracle.MODE_REPLAY, dts=seg, t=t, tau_B2=tau_B2)
        x, t = o["x"], o["t"]
        oE += list(o["diag"][:, 2])
        omin += list(o["diag"][:, 6])
        err = float(np.abs(E[s0:s0 + len(seg)] - o["diag"][:, 2]).max() / E[0])
        banner(f"  oracle replay to step {s0 + len(seg)}: E_M difference in these steps {err:.2e}")
    oE = np.array(oE)
    k_min = int(np.argmin(E))
    dE = np.abs(E - oE) / E[0]
    banner(f"  {len(diag)} steps; E_M minimum at step {k_min} (oracle {int(np.argmin(oE))}); E_M difference "
           f"up to it {dE[:k_min + 1].max():.2e}, at the last step {dE[-1]:.2e}; final min det GPU "
           f"{diag[-1]['min_det']:.3e} oracle {omin[-1]:.3e}")
    assert dE[:k_min + 1].max() < 1e-9
    assert int(np.argmin(oE)) == k_min and k_min < len(diag) - 1
    assert E[-1] > E[k_min] and oE[-1] > oE[k_min]
    assert diag[-1]["min_det"] < 1e-4 and omin[-1] < 1e-4
    assert rel(omin[-1], diag[-1]["min_det"]) < 0.05
