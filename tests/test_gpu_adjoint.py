"""Reverse-mode gradients of the relaxation step (relax_backward) against the oracle.

Reference: the oracle's fixed-dt trajectory in complex arithmetic gives exact directional
derivatives (complex step, Im f(p + i e v) / e with e = 1e-30).  Tolerance: relative 1e-10 of
the directional derivative, scaled by |grad| |v| (cancellation among node contributions).
At the full 64 x 64 x 192 braid size: 40 steps (checkpoints every 10) against complex step
along 2 directions, and 200 steps (checkpoints every 20) against fourth-order central
differences of the GPU forward pass along 32 directions; both measured against the typical
directional derivative |grad| / sqrt(dim) of a random unit direction (1e-10 and 1e-6)."""
import math

import numpy as np
import pytest

import oracle
import paper_1405_0942_amd as R
import workloads as W
from gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

CASES = [
    ("lt_10x9x8", (10, 9, 8), [(-1.0, 1.0), (-0.9, 0.9), (-0.8, 0.8)], (0, 0, 0)),
    ("pxy_12x10x9", (12, 10, 9), [(-1.0, 1.0), (-1.0, 1.0), (-1.0, 1.0)], (1, 1, 0)),
    ("pall_8x9x10", (8, 9, 10), [(0.0, 1.0), (0.0, 1.1), (0.0, 1.2)], (1, 1, 1)),
    ("pz_70x6x7", (70, 6, 7), [(0.0, 3.0), (0.0, 0.5), (0.0, 0.6)], (0, 0, 1)),
]


def make(case, seed=0):
    name, n, spans, bc = case
    g = W.make_grid(n, spans, bc)
    x0 = W.distorted_grid(g, 0.03 * min(g.h), seed=300 + seed)
    B0 = W.smooth_random_field(g, 0.5, seed=400 + seed) + np.array([0.1, 0.2, 1.0])[:, None, None, None]
    return g, x0, B0


def gpu_grad(g, x0, B0, K, dt, seed_EM=1.0, seed_R2=0.0, every=2):
    cfg = R.make_config(g, dt0=dt, adaptive=False, record=True, checkpoint_every=every)
    with R.Relaxation(cfg, dev(x0), dev(B0), K_record=max(K, 1)) as r:
        if K:
            r.step(K, diag=False)
        d = r.diagnostics()
        gx, gb = r.backward(seed_EM, seed_R2)
    return host(gx), host(gb), d


def step_for(g, x0, B0, frac=0.02):
    umax = np.abs(oracle.fields(g, x0, B0)["u"]).max()
    return float(frac * min(g.h) / umax)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("which", ["E_M", "R2"])
def test_gradient_vs_complex_step(case, which):
    banner(f"adjoint vs complex step {case[0]} {which}")
    g, x0, B0 = make(case)
    dt = step_for(g, x0, B0)
    K = 5
    sE, sR = (1.0, 0.0) if which == "E_M" else (0.0, 1.0)
    gx, gb, _ = gpu_grad(g, x0, B0, K, dt, sE, sR, every=2)
    rng = np.random.default_rng(7)
    for _ in range(3):
        vx, vb = rng.standard_normal(x0.shape), rng.standard_normal(B0.shape)
        eps = 1e-30
        E, R2 = oracle.run_fixed_complex(g, x0 + 1j * eps * vx, B0 + 1j * eps * vb, [dt] * K)
        ref = (E if which == "E_M" else R2).imag / eps
        got = float((gx * vx).sum() + (gb * vb).sum())
        scale = math.sqrt((gx ** 2).sum() * (vx ** 2).sum()) + math.sqrt((gb ** 2).sum() * (vb ** 2).sum())
        assert abs(got - ref) <= 1e-10 * scale, (got, ref, scale)


@pytest.mark.parametrize("case", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_seed_only_K0(case):
    """K = 0: closed forms.  E_M is homogeneous of degree 2 in B0: <dE/dB0, B0> = 2 E."""
    banner(f"adjoint K=0 {case[0]}")
    g, x0, B0 = make(case)
    gx, gb, d = gpu_grad(g, x0, B0, 0, 1e-3)
    assert (gb * B0).sum() == pytest.approx(2 * d["E_M"], rel=1e-12)
    eps = 1e-30
    vx = np.random.default_rng(3).standard_normal(x0.shape)
    E, _ = oracle.run_fixed_complex(g, x0 + 1j * eps * vx, B0, [])
    assert float((gx * vx).sum()) == pytest.approx(E.imag / eps, rel=1e-10, abs=1e-12 * np.abs(gx).sum())


def test_translation_invariance_and_checkpoint_interval():
    banner("adjoint translation invariance, checkpoint interval")
    g, x0, B0 = make(CASES[1])
    dt = step_for(g, x0, B0)
    a = gpu_grad(g, x0, B0, 7, dt, every=3)
    b = gpu_grad(g, x0, B0, 7, dt, every=7)
    c = gpu_grad(g, x0, B0, 7, dt, every=1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    # translating every node leaves u and E_M unchanged
    s = a[0].reshape(3, -1).sum(axis=1)
    assert np.abs(s).max() <= 1e-12 * np.abs(a[0]).sum()


def test_autograd_function():
    banner("torch.autograd.Function")
    g, x0, B0 = make(CASES[0])
    dt = step_for(g, x0, B0)
    cfg = R.make_config(g, dt0=dt, adaptive=False, record=True, checkpoint_every=2)
    xt = dev(x0).requires_grad_(True)
    bt = dev(B0).requires_grad_(True)
    E, R2 = R.relax_energy(xt, bt, cfg, 4)
    (2.0 * E + 3.0 * R2).backward()
    gx_e, gb_e, _ = gpu_grad(g, x0, B0, 4, dt, 1.0, 0.0)
    gx_r, gb_r, _ = gpu_grad(g, x0, B0, 4, dt, 0.0, 1.0)
    assert np.allclose(host(xt.grad), 2 * gx_e + 3 * gx_r, rtol=1e-12, atol=1e-14 * np.abs(gx_e).max())
    assert np.allclose(host(bt.grad), 2 * gb_e + 3 * gb_r, rtol=1e-12, atol=1e-14 * np.abs(gb_e).max())


def _joint_scale(gx, gb):
    """|g| |v| / sqrt(dim) for unit v: the size of a typical directional derivative along a
    random unit direction in the joint (x0, B0) space.  Errors are measured against it (a
    single direction's derivative can be arbitrarily close to zero)."""
    return float(np.sqrt((gx ** 2).sum() + (gb ** 2).sum()) / np.sqrt(gx.size + gb.size))


def test_braid_full_size_complex_step():
    """64 x 64 x 192 braid, twist amplitudes U(0.5, 1.5) (seed 4), 40 fixed-dt steps with
    checkpoints every 10 (four segments, every z-chunk seam of the launch): directional
    derivatives of E_M(x_40) against the oracle's complex-step derivative along 2 seeded unit
    directions (1e-10 of the typical directional derivative)."""
    banner("adjoint braid 64x64x192, 40 steps, vs complex step (2 directions)")
    w = W.braid(64, 192, seed=4)
    g = w.grid
    dt, K = 2e-3, 40
    gx, gb, _ = gpu_grad(g, w.x0, w.B0, K, dt, every=10)
    scale = _joint_scale(gx, gb)
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(2):
        vx, vb = rng.standard_normal(w.x0.shape), rng.standard_normal(w.B0.shape)
        n = np.sqrt((vx ** 2).sum() + (vb ** 2).sum())
        vx, vb = vx / n, vb / n
        eps = 1e-30
        Ez, _ = oracle.run_fixed_complex(g, w.x0 + 1j * eps * vx, w.B0 + 1j * eps * vb, np.full(K, dt))
        cs = Ez.imag / eps
        got = float((gx * vx).sum() + (gb * vb).sum())
        worst = max(worst, abs(got - cs) / scale)
        assert abs(got - cs) < 1e-10 * scale, (got, cs, scale)
    banner(f"  worst difference {worst:.2e} of the typical directional derivative {scale:.3e}")


def test_braid_full_size_central_differences():
    """64 x 64 x 192 braid, twist amplitudes U(0.5, 1.5) (seed 4), 200 fixed-dt steps with
    checkpoints every 20: directional derivatives of E_M(x_200) against fourth-order central
    differences of the GPU forward pass along 32 seeded unit Gaussian directions in the joint
    (x0, B0) space (1e-6 of the typical directional derivative; the differences are limited
    by the rounding of E_M, about 1e-12 of its value)."""
    banner("adjoint braid 64x64x192, 200 steps, vs central differences (32 directions)")
    w = W.braid(64, 192, seed=4)
    g = w.grid
    dt, K = 2e-3, 200
    gx, gb, d = gpu_grad(g, w.x0, w.B0, K, dt, every=20)
    scale = _joint_scale(gx, gb)
    cfg = R.make_config(g, dt0=dt, adaptive=False)
    x0d, b0d = dev(w.x0), dev(w.B0)
    gxd, gbd = dev(gx), dev(gb)

    def energy(vx, vb, h):
        with R.Relaxation(cfg, (x0d + h * vx).contiguous(), (b0d + h * vb).contiguous()) as r:
            r.step(K, diag=False)
            return r.diagnostics()["E_M"]
    gen = torch.Generator(device="cuda").manual_seed(4)
    worst = 0.0
    for _ in range(32):
        vx = torch.randn(x0d.shape, generator=gen, device="cuda", dtype=torch.float64)
        vb = torch.randn(b0d.shape, generator=gen, device="cuda", dtype=torch.float64)
        nrm = float(torch.sqrt((vx * vx).sum() + (vb * vb).sum()))
        vx, vb = vx / nrm, vb / nrm
        h = 2e-2  # about 1e-6 |(x0, B0)| / |v| (|(x0, B0)| is about 1.3e4)
        d1 = energy(vx, vb, h) - energy(vx, vb, -h)
        d2 = energy(vx, vb, 2 * h) - energy(vx, vb, -2 * h)
        fd = (8 * d1 - d2) / (12 * h)
        got = float((gxd * vx).sum() + (gbd * vb).sum())
        worst = max(worst, abs(got - fd) / scale)
        assert abs(got - fd) < 1e-6 * scale, (got, fd, scale)
    banner(f"  worst difference {worst:.2e} of the typical directional derivative {scale:.3e}")
