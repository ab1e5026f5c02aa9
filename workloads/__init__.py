"""Seeded synthetic inputs for the relaxation workloads.

This module only builds inputs: reference grids, initial fields B0(X) and initial
positions x0(X).  It holds none of the relaxation arithmetic (no Jacobian, no
pull-back, no curl, no time stepping), so both the CPU oracle and the HIP path
can take their inputs from here without sharing any of the method.

Layout of every field: float64 numpy array of shape (3, nz, ny, nx), i.e. the
component index first and x fastest in memory (structure of arrays).

Grids are node-centred.  Along a line-tied axis the two end points are boundary
nodes (a "vertex grid", h = L/(n-1)); along a periodic axis there are n nodes and
the period is n*h, with no duplicated end point (the paper's periodic ghost
convention, Sec. 2.5 "Boundary Conditions").

Field recipes (all divergence-free):
  * twist region (the paper's Pontin09 form, Sec. 3.1, eq. "B init Pontin09"):
        s * (2k/a) exp(-((X-cx)^2+Y^2)/a^2 - (Z-zc)^2/l^2) * (-Y, X-cx, 0)
  * IsoHelix (Sec. 3.1, eq. "B init analytical") and its closed-form relaxed
    map (eq. "x analytical relaxed"),
  * ABC Beltrami field (A=B=C=1).
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

LINE_TIED = 0
PERIODIC = 1


@dataclasses.dataclass(frozen=True)
class Grid:
    """Logically rectangular reference grid X_ijk = origin + (i hx, j hy, k hz)."""

    n: tuple  # (nx, ny, nz)
    h: tuple  # (hx, hy, hz)
    bc: tuple  # per axis LINE_TIED / PERIODIC
    origin: tuple = (0.0, 0.0, 0.0)

    @property
    def N(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def shape(self) -> tuple:
        """numpy shape of one field: (3, nz, ny, nx)."""
        return (3, self.n[2], self.n[1], self.n[0])

    def axes(self):
        """1-D node coordinates along x, y, z."""
        return [self.origin[a] + self.h[a] * np.arange(self.n[a], dtype=np.float64) for a in range(3)]

    def coords(self):
        """Broadcast-ready X, Y, Z of shape (nz, ny, nx)."""
        xs, ys, zs = self.axes()
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        return X, Y, Z

    def identity(self) -> np.ndarray:
        """x = X (the undistorted grid) as a (3, nz, ny, nx) array."""
        X, Y, Z = self.coords()
        return np.ascontiguousarray(np.stack([X, Y, Z]))

    def lengths(self):
        """Domain extent per axis: (n-1)h line-tied, n h periodic."""
        return tuple((self.n[a] - 1) * self.h[a] if self.bc[a] == LINE_TIED else self.n[a] * self.h[a]
                     for a in range(3))


def vertex_axis(lo: float, hi: float, n: int):
    """(origin, spacing) of a line-tied axis with both end points on the grid."""
    return lo, (hi - lo) / (n - 1)


def periodic_axis(lo: float, hi: float, n: int):
    """(origin, spacing) of a periodic axis of period hi-lo with n nodes."""
    return lo, (hi - lo) / n


def make_grid(n, spans, bc) -> Grid:
    origin, h = [], []
    for a in range(3):
        lo, hi = spans[a]
        o, d = vertex_axis(lo, hi, n[a]) if bc[a] == LINE_TIED else periodic_axis(lo, hi, n[a])
        origin.append(o)
        h.append(d)
    return Grid(tuple(int(v) for v in n), tuple(h), tuple(int(b) for b in bc), tuple(origin))


# ----------------------------------------------------------------------------------------
# Initial fields B0(X)
# ----------------------------------------------------------------------------------------

def uniform_field(g: Grid, b=(0.0, 0.0, 1.0)) -> np.ndarray:
    out = np.empty(g.shape)
    for c in range(3):
        out[c] = b[c]
    return out


def twist_region(X, Y, Z, k, a, l, cx=0.0, zc=0.0, s=1.0):
    """One twist region s*(2k/a) exp(-((X-cx)^2+Y^2)/a^2-(Z-zc)^2/l^2) (-Y, X-cx, 0)."""
    amp = s * (2.0 * k / a) * np.exp(-((X - cx) ** 2 + Y ** 2) / a ** 2 - (Z - zc) ** 2 / l ** 2)
    return -Y * amp, (X - cx) * amp


def single_twist_field(g: Grid, k=1.0, a=0.5, l=0.5, s=1.0) -> np.ndarray:
    """e_z + one twist region centred on the origin."""
    X, Y, Z = g.coords()
    bx, by = twist_region(X, Y, Z, k, a, l, 0.0, 0.0, s)
    return np.ascontiguousarray(np.stack([bx, by, np.ones_like(X)]))


def braid_field(g: Grid, ks=(1.0,) * 6, a=math.sqrt(2.0), l=2.0, periods=None, images=1) -> np.ndarray:
    """e_z + 6 twist regions at z_m = -15 + 6m, centre x = (-1)^m, sign (-1)^m.

    Along periodic x / y the Gaussians are summed over the images shifted by
    multiples of the period (|m_x|, |m_y| <= images) so that B0 is continuous
    across the seam; a sum of divergence-free terms stays divergence-free.
    """
    X, Y, Z = g.coords()
    Lx, Ly, _ = g.lengths() if periods is None else periods
    sx = range(-images, images + 1) if g.bc[0] == PERIODIC else [0]
    sy = range(-images, images + 1) if g.bc[1] == PERIODIC else [0]
    bx = np.zeros_like(X)
    by = np.zeros_like(X)
    for m in range(6):
        zc = -15.0 + 6.0 * m
        cx = float((-1) ** m)
        s = float((-1) ** m)
        for ix in sx:
            for iy in sy:
                tx, ty = twist_region(X - ix * Lx, Y - iy * Ly, Z, ks[m], a, l, cx, zc, s)
                bx += tx
                by += ty
    return np.ascontiguousarray(np.stack([bx, by, np.ones_like(X)]))


def isohelix_field(g: Grid, phi=math.pi / 4, B0=1.0, ar=math.sqrt(2.0), az=2.0) -> np.ndarray:
    """IsoHelix initial field (Sec. 3.1): (2 B0 Z / az^2) e^{...} phi (Y, -X, 0) + B0 e_z."""
    X, Y, Z = g.coords()
    amp = (2.0 * B0 * Z / az ** 2) * np.exp(-(X ** 2 + Y ** 2) / ar ** 2 - Z ** 2 / az ** 2) * phi
    return np.ascontiguousarray(np.stack([Y * amp, -X * amp, B0 * np.ones_like(X)]))


def pontin09_field(g: Grid, phis=(math.pi, -math.pi), Ls=(-5.0, 5.0), B0=1.0, ar=math.sqrt(2.0),
                   az=2.0) -> np.ndarray:
    """Pontin09 initial field (Sec. 3.1, eq. "B init Pontin09"): B0 e_z plus two twist regions
    (2 B0 phi_i / (pi a_r)) e^{-(X^2+Y^2)/a_r^2 - (Z-L_i)^2/a_z^2} (-Y, X, 0) centred at
    Z = L_i.  The paper does not give L_i; the default puts them half way to the ends of the
    [-10, 10] box."""
    X, Y, Z = g.coords()
    bx = np.zeros_like(X)
    by = np.zeros_like(X)
    for phi, L in zip(phis, Ls):
        amp = (2.0 * B0 * phi / (math.pi * ar)) * np.exp(-(X ** 2 + Y ** 2) / ar ** 2 - (Z - L) ** 2 / az ** 2)
        bx += -Y * amp
        by += X * amp
    return np.ascontiguousarray(np.stack([bx, by, B0 * np.ones_like(X)]))


def isohelix_relaxed_map(g: Grid, phi=math.pi / 4, ar=math.sqrt(2.0), az=2.0) -> np.ndarray:
    """Closed-form relaxed positions of the IsoHelix field (Sec. 3.1, eq. "x analytical relaxed")."""
    X, Y, Z = g.coords()
    th = np.exp(-(X ** 2 + Y ** 2) / ar ** 2 - Z ** 2 / az ** 2) * phi
    c, s = np.cos(th), np.sin(th)
    return np.ascontiguousarray(np.stack([c * X + s * Y, c * Y - s * X, Z]))


def abc_field(g: Grid, A=1.0, B=1.0, C=1.0) -> np.ndarray:
    """ABC Beltrami field (A sin Z + C cos Y, B sin X + A cos Z, C sin Y + B cos X)."""
    X, Y, Z = g.coords()
    return np.ascontiguousarray(np.stack([A * np.sin(Z) + C * np.cos(Y),
                                          B * np.sin(X) + A * np.cos(Z),
                                          C * np.sin(Y) + B * np.cos(X)]))


# ----------------------------------------------------------------------------------------
# Initial positions x0(X) = X + d(X)
# ----------------------------------------------------------------------------------------

def _scale_to_max_norm(d: np.ndarray, amp: float) -> np.ndarray:
    m = float(np.sqrt((d ** 2).sum(axis=0)).max())
    return d * (amp / m) if m > 0 else d


def wall_sine_displacement(g: Grid, amp: float, seed: int, modes=(1, 2), lo=-1.0, hi=1.0) -> np.ndarray:
    """d_c = sum_{m in modes^3} alpha_{c,m} prod_a sin(m_a pi (X_a-lo)/(hi-lo)), alpha ~ N(0,1).

    Vanishes on every wall of the box [lo,hi]^3; scaled so that max_nodes |d| = amp.
    """
    rng = np.random.default_rng(seed)
    X, Y, Z = g.coords()
    L = hi - lo
    d = np.zeros(g.shape)
    for c in range(3):
        for m in itertools.product(modes, repeat=3):
            alpha = rng.standard_normal()
            d[c] += alpha * (np.sin(m[0] * math.pi * (X - lo) / L) * np.sin(m[1] * math.pi * (Y - lo) / L)
                             * np.sin(m[2] * math.pi * (Z - lo) / L))
    return _scale_to_max_norm(d, amp)


def fourier_modes(kmax: int = 3):
    """One representative k of every +/- pair of integer vectors with 0 < |k| <= kmax."""
    out = []
    for k in itertools.product(range(-kmax, kmax + 1), repeat=3):
        if 0 < k[0] ** 2 + k[1] ** 2 + k[2] ** 2 <= kmax ** 2 and k > (0, 0, 0):
            out.append(k)
    return out


def fourier_displacement(g: Grid, amp: float, seed: int, kmax: int = 3) -> np.ndarray:
    """Divergence-free periodic displacement sum_k (alpha_k cos k.X + beta_k sin k.X).

    alpha_k, beta_k are standard Gaussian 3-vectors projected perpendicular to k.
    The box must be periodic with period 2 pi on every axis.  Evaluated by an
    inverse FFT of the placed coefficients; scaled so that max_nodes |d| = amp.
    """
    assert all(b == PERIODIC for b in g.bc)
    rng = np.random.default_rng(seed)
    nx, ny, nz = g.n
    spec = np.zeros((3, nz, ny, nx), dtype=np.complex128)
    for k in fourier_modes(kmax):
        kv = np.array(k, dtype=np.float64)
        al = rng.standard_normal(3)
        be = rng.standard_normal(3)
        al -= kv * (al @ kv) / (kv @ kv)
        be -= kv * (be @ kv) / (kv @ kv)
        # alpha cos(k.X) + beta sin(k.X) = Re[(alpha - i beta) e^{i k.X}]
        #                                = (c e^{ikX} + conj(c) e^{-ikX}) / 2, c = alpha - i beta
        cpos = 0.5 * (al - 1j * be)
        for sgn, cc in ((1, cpos), (-1, np.conj(cpos))):
            ix, iy, iz = (sgn * k[0]) % nx, (sgn * k[1]) % ny, (sgn * k[2]) % nz
            spec[:, iz, iy, ix] += cc
    # d(X) at X_j = origin + j h with h = 2 pi / n: sum_k c_k e^{i k X}
    X0 = g.origin
    phase = [np.exp(1j * np.fft.fftfreq(g.n[a], 1.0 / g.n[a]) * X0[a]) for a in range(3)]
    spec *= phase[2][None, :, None, None] * phase[1][None, None, :, None] * phase[0][None, None, None, :]
    d = np.fft.ifftn(spec, axes=(1, 2, 3)).real * (nx * ny * nz)
    return _scale_to_max_norm(np.ascontiguousarray(d), amp)


# ----------------------------------------------------------------------------------------
# The five named workloads
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    x0: np.ndarray
    B0: np.ndarray
    steps: int
    tol: float
    dt0: float
    note: str = ""


def single_twist_16(seed: int = 1) -> Workload:
    """16^3 on [-1,1]^3, all faces line-tied; one twist region; x0 = X + smooth wall-free d (max 0.02)."""
    g = make_grid((16, 16, 16), [(-1.0, 1.0)] * 3, (LINE_TIED,) * 3)
    B0 = single_twist_field(g, k=1.0, a=0.5, l=0.5, s=1.0)
    x0 = g.identity() + wall_sine_displacement(g, 0.02, seed)
    return Workload("single_twist_16^3", g, x0, B0, steps=100, tol=1e-8, dt0=1e-3)


def braid_grid(nx: int, nz: int) -> Grid:
    return make_grid((nx, nx, nz), [(-4.0, 4.0), (-4.0, 4.0), (-24.0, 24.0)], (PERIODIC, PERIODIC, LINE_TIED))


def braid(nx: int = 64, nz: int = 192, ks=None, seed: int | None = None) -> Workload:
    """Six-twist braid on [-4,4]^2 x [-24,24]: periodic x, y; line-tied z; x0 = X."""
    g = braid_grid(nx, nz)
    if ks is None and seed is not None:
        ks = tuple(np.random.default_rng(seed).uniform(0.5, 1.5, 6))
    ks = ks if ks is not None else (1.0,) * 6
    B0 = braid_field(g, ks=ks)
    return Workload(f"braid_{nx}x{nx}x{nz}", g, g.identity(), B0, steps=10_000, tol=1e-7, dt0=1e-3,
                    note=f"twist amplitudes {tuple(float(k) for k in ks)}")


def abc_box(n: int = 256, seed: int = 5, amp: float = 0.1) -> Workload:
    """ABC field on the periodic box [0, 2 pi)^3 with a divergence-free |k|<=3 displacement of x."""
    g = make_grid((n, n, n), [(0.0, 2 * math.pi)] * 3, (PERIODIC,) * 3)
    B0 = abc_field(g)
    x0 = g.identity() + fourier_displacement(g, amp, seed)
    return Workload(f"abc_{n}^3", g, x0, B0, steps=200, tol=1e-7, dt0=1e-3)


# ----------------------------------------------------------------------------------------
# Generic seeded inputs for operator tests
# ----------------------------------------------------------------------------------------

def checkerboard_bump(g: Grid, amp_rel: float, width: float) -> np.ndarray:
    """x-displacement (-1)^(i+j+k) amp_rel h_x exp(-|idx - centre|^2 / width^2) (index units).

    Central differences of a checkerboard cancel, so det F stays near 1 while the edges to
    neighbours flip once amp_rel exceeds 1/2: concave cells inside a smooth grid."""
    nx, ny, nz = g.n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = np.where((i + j + k) % 2 == 0, 1.0, -1.0)
    r2 = ((i - nx / 2) ** 2 + (j - ny / 2) ** 2 + (k - nz / 2) ** 2) / width ** 2
    d = np.zeros(g.shape)
    d[0] = amp_rel * g.h[0] * c * np.exp(-r2)
    return d


def smooth_random_field(g: Grid, amp: float, seed: int, mmax: int = 2) -> np.ndarray:
    """Sum of random low-order cosine modes, periodic along periodic axes.

    d_c = sum_m alpha_{c,m} cos(2 pi m . xi + phase_{c,m}), xi_a = (X_a - origin_a)/L_a with
    L_a the period (periodic axis) or the domain length (line-tied axis); scaled so that
    max_nodes |d| = amp.
    """
    rng = np.random.default_rng(seed)
    X, Y, Z = g.coords()
    L = g.lengths()
    xi = [(X - g.origin[0]) / L[0], (Y - g.origin[1]) / L[1], (Z - g.origin[2]) / L[2]]
    d = np.zeros(g.shape)
    for c in range(3):
        for m in itertools.product(range(mmax + 1), repeat=3):
            if m == (0, 0, 0):
                continue
            arg = 2 * math.pi * (m[0] * xi[0] + m[1] * xi[1] + m[2] * xi[2]) + rng.uniform(0, 2 * math.pi)
            d[c] += rng.standard_normal() * np.cos(arg)
    return _scale_to_max_norm(d, amp)


def distorted_grid(g: Grid, amp: float, seed: int) -> np.ndarray:
    """x0 = X + a smooth random displacement of maximum length amp."""
    return g.identity() + smooth_random_field(g, amp, seed)
