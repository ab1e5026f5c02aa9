"""Helpers shared by the GPU tests: device tensors, running the HIP path, comparisons."""
import numpy as np

import paper_1405_0942_amd as R


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def nrel(a, b):
    """normwise relative error ||a-b||_inf / ||b||_inf"""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def context(grid, x0, B0, K_record=0, **cfg_kw):
    cfg = R.make_config(grid, **cfg_kw)
    return R.Relaxation(cfg, dev(x0), dev(B0), K_record=K_record)


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def nrel_inc(x1, x0, xo1):
    """Normwise relative error of the increment x1 - x0 against the oracle's xo1 - x0, up to the
    rounding of the stored positions: a node may differ by one unit in the last place of its
    stored coordinate (two sums that agree to a few ulps of the increment can still round the
    position to neighbouring doubles), which is removed before the norm is taken."""
    x1, x0, xo1 = (np.asarray(a, dtype=np.float64) for a in (x1, x0, xo1))
    d = np.abs((x1 - x0) - (xo1 - x0))
    ulp = np.spacing(np.maximum(np.abs(x1), np.abs(xo1)))
    return float(np.maximum(d - ulp, 0.0).max() / max(np.abs(xo1 - x0).max(), 1e-300))
