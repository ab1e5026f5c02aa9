"""IsoHelix (and Pontin09) set-ups and the diagnostics of their relaxed states (Sec. 3.1,
3.2), shared by the oracle pins and the GPU accuracy and breakdown runs.

  sigma_B = sqrt(sum |B - B_relax|^2 / N), B_relax = e_z            (eq. "B relaxed"),
  sigma_x = sqrt(sum |x - x_relax|^2 / N), x_relax the rotated grid (eq. "x analytical relaxed"),
  eps*    = max over pairs of central-line nodes of a_r |alpha*_i - alpha*_j| / |X_i - X_j|,
            alpha* = J.B / B^2, on X = Y = 0 (eq. "epsilon star"; the interior nodes of the line).
"""
import math
import os

import numpy as np

import workloads as W

PHI = math.pi / 4
AR = math.sqrt(2.0)
HERE = os.path.dirname(os.path.abspath(__file__))


def grid(n):
    """n^3 vertex grid over [-4, 4]^2 x [-10, 10], all faces line-tied (n odd: a node on X = Y = 0)."""
    return W.make_grid((n, n, n), [(-4.0, 4.0), (-4.0, 4.0), (-10.0, 10.0)], (0, 0, 0))


PHIS = {"pi/4": math.pi / 4, "pi/2": math.pi / 2, "pi": math.pi}


def table1(phi="pi/4"):
    """{n: (xi, eps*, sigma_B, sigma_x), or None for a run that did not converge} as the paper
    prints them (Table 1, mimetic rows of twist angle phi: "pi/4", "pi/2" or "pi")."""
    out = {}
    with open(os.path.join(HERE, "golden", "isohelix_table1_mimetic.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = line.split()
                if v[0] == phi:
                    out[int(v[1])] = None if v[2] == "--" else tuple(float(a) for a in v[2:])
    return out


def table2():
    """{n: (xi, eps*)} as the paper prints them (Table 2: Pontin09, mimetic, phi = pi/2)."""
    out = {}
    with open(os.path.join(HERE, "golden", "pontin09_table2_mimetic_pi2.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = line.split()
                out[int(v[0])] = tuple(float(a) for a in v[1:])
    return out


def relaxed_state_errors(g, x, B, J, phi=PHI):
    """(sigma_B, sigma_x, eps*) of positions x with field B and current J (IsoHelix of twist
    angle phi)."""
    N = g.N
    sB = math.sqrt(float(((B - np.array([0.0, 0.0, 1.0])[:, None, None, None]) ** 2).sum()) / N)
    sx = math.sqrt(float(((x - W.isohelix_relaxed_map(g, phi)) ** 2).sum()) / N)
    alpha = (J * B).sum(axis=0) / (B * B).sum(axis=0)
    return sB, sx, epsilon_star(g, alpha)


def epsilon_star(g, alpha, a_r=AR):
    """eps* of an alpha* map (nz, ny, nx): the largest a_r |alpha*_i - alpha*_j| / |Z_i - Z_j|
    over pairs of interior nodes of the central line X = Y = 0 (eq. "epsilon star")."""
    nx, ny, nz = g.n
    i, j = (nx - 1) // 2, (ny - 1) // 2
    al = alpha[1:nz - 1, j, i]
    Z = g.origin[2] + g.h[2] * np.arange(1, nz - 1)
    dA = np.abs(al[:, None] - al[None, :])
    dZ = np.abs(Z[:, None] - Z[None, :])
    np.fill_diagonal(dZ, np.inf)
    return float(a_r * (dA / dZ).max())
