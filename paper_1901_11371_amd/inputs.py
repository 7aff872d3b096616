"""Seeded synthetic inputs for the 2D TM-EFIE workloads (open PEC curves).

This module only makes inputs: curve node arrays, incidence angles, plane-wave
excitations, impedance values and random vectors.  It holds none of the
method's arithmetic (no kernel entries, no compression, no solves) and is the
one module shared by the CPU oracle and the GPU library.

Geometry conventions (the paper, Sec. 3.1: pulse basis on line segments with
centre rho_i and length w_i; Sec. 4: synthetic analytic open curves):

* wavelength 1, wavenumber kappa = 2*pi;
* 10 segments per wavelength, so a curve carrying N segments has arc length
  N/10;
* N+1 nodes at equal arc length along the analytic curve; segment i is the
  chord between nodes i and i+1 (curve-parameter order, which is the geometric
  ordering the paper requires, Sec. 3.1 and Sec. 3.3.1);
* several curves are concatenated in generation order.

Every random draw uses ``numpy.random.default_rng(SEED_BASE + workload_index)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 190111371
KAPPA = 2.0 * math.pi          # wavelength 1
ETA0 = 376.730313668           # free-space impedance in ohms
SEGMENTS_PER_WAVELENGTH = 10.0


@dataclass
class Curves:
    """Nodes of one or more open polylines.

    ``xy`` holds the nodes of all curves, shape (total_nodes, 2), float64;
    curve c owns nodes ``xy[node_off[c]:node_off[c+1]]`` and contributes
    ``node_off[c+1] - node_off[c] - 1`` segments.
    """
    xy: np.ndarray
    node_off: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_segments(self) -> int:
        return int(self.node_off[-1] - len(self.node_off) + 1)

    @property
    def ncurves(self) -> int:
        return len(self.node_off) - 1


def _single(xy: np.ndarray, name: str, **meta) -> Curves:
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    return Curves(xy, np.array([0, xy.shape[0]], dtype=np.int64), name, dict(meta))


def _invert_monotone(F, dF, targets, t0, t1, iters=60):
    """Solve F(t) = target for a monotone increasing F on [t0, t1] (Newton with
    bisection safeguard), vectorised over targets."""
    lo = np.full_like(targets, t0)
    hi = np.full_like(targets, t1)
    # initial guess: linear interpolation between the ends
    F0, F1 = F(np.array([t0]))[0], F(np.array([t1]))[0]
    t = t0 + (targets - F0) / (F1 - F0) * (t1 - t0)
    for _ in range(iters):
        f = F(t) - targets
        lo = np.where(f < 0, t, lo)
        hi = np.where(f >= 0, t, hi)
        step = f / dF(t)
        tn = t - step
        bad = (tn <= lo) | (tn >= hi) | ~np.isfinite(tn)
        tn = np.where(bad, 0.5 * (lo + hi), tn)
        if np.max(np.abs(tn - t)) <= 1e-15 * max(1.0, abs(t1)):
            t = tn
            break
        t = tn
    return t


def strip(n: int, origin=(0.0, 0.0), angle: float = 0.0) -> Curves:
    """Straight strip of n segments of length 1/10 starting at ``origin``."""
    s = np.arange(n + 1, dtype=np.float64) * (1.0 / SEGMENTS_PER_WAVELENGTH)
    xy = np.stack([origin[0] + s * math.cos(angle), origin[1] + s * math.sin(angle)], axis=1)
    return _single(xy, "strip", length=n / SEGMENTS_PER_WAVELENGTH)


def circular_arc(n: int, radius: float, theta0: float, theta1: float, center=(0.0, 0.0)) -> Curves:
    """Arc of a circle (angles theta0 -> theta1) with n equal-arc-length segments."""
    th = theta0 + (theta1 - theta0) * np.arange(n + 1, dtype=np.float64) / n
    xy = np.stack([center[0] + radius * np.cos(th), center[1] + radius * np.sin(th)], axis=1)
    return _single(xy, "arc", radius=radius)


def semicircle(n: int) -> Curves:
    """Semicircle of arc length n/10 (radius = length/pi)."""
    length = n / SEGMENTS_PER_WAVELENGTH
    c = circular_arc(n, length / math.pi, 0.0, math.pi)
    c.name = "semicircle"
    return c


def parabola(n: int) -> Curves:
    """Parabolic arc y = 0.3 x^2 / Lp, x in [-Lp/2, Lp/2], of arc length n/10."""
    length = n / SEGMENTS_PER_WAVELENGTH
    # arc length of y = c x^2 over [-Lp/2, Lp/2] is Lp * g with c = 0.3/Lp:
    # with u = 2 c x, ds = sqrt(1+u^2) dx; over the whole arc u runs in [-0.3, 0.3].
    umax = 0.3
    g = (umax * math.sqrt(1 + umax * umax) + math.asinh(umax)) / (2 * umax)
    Lp = length / g
    c = 0.3 / Lp

    def arc(x):  # arc length from x = -Lp/2
        u = 2 * c * x
        prim = (u * np.sqrt(1 + u * u) + np.arcsinh(u)) / (4 * c)
        u0 = -umax
        prim0 = (u0 * math.sqrt(1 + u0 * u0) + math.asinh(u0)) / (4 * c)
        return prim - prim0

    def darc(x):
        return np.sqrt(1 + (2 * c * x) ** 2)

    targets = np.arange(n + 1, dtype=np.float64) * (length / n)
    x = _invert_monotone(arc, darc, targets, -Lp / 2, Lp / 2)
    x[0], x[-1] = -Lp / 2, Lp / 2
    xy = np.stack([x, c * x * x], axis=1)
    return _single(xy, "parabola", Lp=Lp)


def archimedean_spiral(n: int, theta0: float = math.pi, theta1: float = 6 * math.pi) -> Curves:
    """Spiral r = a*theta, theta in [theta0, theta1], of arc length n/10."""
    length = n / SEGMENTS_PER_WAVELENGTH

    def prim(t):  # integral of sqrt(1 + t^2)
        return 0.5 * (t * np.sqrt(1 + t * t) + np.arcsinh(t))

    unit = float(prim(np.array([theta1]))[0] - prim(np.array([theta0]))[0])
    a = length / unit

    def arc(t):
        return a * (prim(t) - prim(np.array([theta0]))[0])

    def darc(t):
        return a * np.sqrt(1 + t * t)

    targets = np.arange(n + 1, dtype=np.float64) * (length / n)
    th = _invert_monotone(arc, darc, targets, theta0, theta1)
    th[0], th[-1] = theta0, theta1
    r = a * th
    xy = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    return _single(xy, "spiral", a=a)


def arc_with_angle(n: int, angle: float) -> Curves:
    """Circular arc of arc length n/10 subtending `angle` (radius = length /
    angle), symmetric about the y axis; the family of the paper's
    arc-angle study (Sec. 4)."""
    length = n / SEGMENTS_PER_WAVELENGTH
    radius = length / angle
    c = circular_arc(n, radius, math.pi / 2 - angle / 2, math.pi / 2 + angle / 2)
    c.name = "arc"
    c.meta["angle"] = angle
    return c


def arc_array(n_total: int, count: int, angle: float = math.pi / 2, gap: float = 2.0) -> Curves:
    """`count` identical circular arcs (each subtending `angle`, n_total /
    count segments) side by side along the x axis, `gap` wavelengths between
    the end of one and the start of the next; the family of the paper's
    arc-array study (Sec. 4).  Curves are concatenated left to right."""
    n = n_total // count
    if n * count != n_total:
        raise ValueError("n_total must be a multiple of count")
    length = n / SEGMENTS_PER_WAVELENGTH
    radius = length / angle
    chord = 2 * radius * math.sin(angle / 2)
    pieces = []
    for k in range(count):
        cx = k * (chord + gap)
        # arc above its chord, endpoints at x = cx - chord/2 and cx + chord/2
        cy = -radius * math.cos(angle / 2)
        pieces.append(circular_arc(n, radius, math.pi / 2 + angle / 2, math.pi / 2 - angle / 2,
                                   center=(cx, cy)).xy)
    node_off = np.zeros(count + 1, dtype=np.int64)
    node_off[1:] = np.cumsum([p.shape[0] for p in pieces])
    return Curves(np.ascontiguousarray(np.concatenate(pieces, axis=0)), node_off, "arc_array",
                  dict(count=count, angle=angle, gap=gap))


def multi_curve(n_total: int, ncurves: int = 8, seed: int | None = None) -> Curves:
    """Disjoint strips (even index) and circular arcs (odd index) of random
    length and orientation, centred on a 4 x 2 grid; segment counts are
    proportional to length and sum to n_total."""
    rng = np.random.default_rng(SEED_BASE + 4 if seed is None else seed)
    rel = rng.uniform(0.5, 2.0, size=ncurves)
    total_len = n_total / SEGMENTS_PER_WAVELENGTH
    lengths = rel / rel.sum() * total_len
    counts = np.floor(lengths / total_len * n_total).astype(np.int64)
    counts[-1] = n_total - counts[:-1].sum()
    lengths = counts / SEGMENTS_PER_WAVELENGTH
    angles = rng.uniform(math.pi / 3, math.pi, size=ncurves)
    orient = rng.uniform(0.0, 2 * math.pi, size=ncurves)
    pitch = 1.1 * float(lengths.max())
    pieces = []
    for c in range(ncurves):
        cx, cy = (c % 4) * pitch, (c // 4) * pitch
        n = int(counts[c])
        if c % 2 == 0:
            half = lengths[c] / 2
            o = (cx - half * math.cos(orient[c]), cy - half * math.sin(orient[c]))
            pieces.append(strip(n, origin=o, angle=float(orient[c])).xy)
        else:
            radius = lengths[c] / angles[c]
            # arc centred so its midpoint sits at the grid centre
            mid = orient[c]
            ccx, ccy = cx - radius * math.cos(mid), cy - radius * math.sin(mid)
            pieces.append(circular_arc(n, radius, mid - angles[c] / 2, mid + angles[c] / 2,
                                       center=(ccx, ccy)).xy)
    node_off = np.zeros(ncurves + 1, dtype=np.int64)
    node_off[1:] = np.cumsum([p.shape[0] for p in pieces])
    return Curves(np.ascontiguousarray(np.concatenate(pieces, axis=0)), node_off, "multi",
                  dict(counts=counts.tolist()))


# --------------------------------------------------------------------------
# excitations, impedances and random vectors
# --------------------------------------------------------------------------

def segment_midpoints(curves: Curves) -> np.ndarray:
    """Midpoints of the chords, in segment order (used to place the incident
    plane wave; the excitation b_i is the incident field at the centre of
    segment i)."""
    mids = []
    for c in range(curves.ncurves):
        p = curves.xy[curves.node_off[c]:curves.node_off[c + 1]]
        mids.append(0.5 * (p[:-1] + p[1:]))
    return np.concatenate(mids, axis=0)


def plane_wave_rhs(curves: Curves, angles, kappa: float = KAPPA) -> np.ndarray:
    """Unit-amplitude incident plane waves exp(-i kappa (x cos phi + y sin phi))
    sampled at the segment centres; returns complex128 of shape (len(angles), N)."""
    rho = segment_midpoints(curves)
    angles = np.atleast_1d(np.asarray(angles, dtype=np.float64))
    ph = kappa * (np.outer(np.cos(angles), rho[:, 0]) + np.outer(np.sin(angles), rho[:, 1]))
    return np.exp(-1j * ph)


def uniform_angles(nrhs: int) -> np.ndarray:
    return 2 * math.pi * np.arange(nrhs, dtype=np.float64) / nrhs


def impedance(n: int, seed: int) -> np.ndarray:
    """Per-unknown surface impedance z_i = u_i (1 + i), u_i ~ U(0, 0.1 eta0)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 0.1 * ETA0, size=n)
    return u * (1 + 1j)


def random_complex(shape, seed: int) -> np.ndarray:
    """(g1 + i g2)/sqrt(2) with standard normal g1, g2."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(size=tuple(np.atleast_1d(shape)) + (2,))
    return (g[..., 0] + 1j * g[..., 1]) / math.sqrt(2.0)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    index: int
    name: str
    curves: Curves
    n0: int
    tol: float
    angles: np.ndarray
    dtype: str
    z: np.ndarray | None = None

    @property
    def seed(self) -> int:
        return SEED_BASE + self.index

    @property
    def n(self) -> int:
        return self.curves.n_segments


def workload(index: int, n: int | None = None, nrhs: int | None = None) -> Workload:
    """The five synthetic workloads (0-based index); ``n``/``nrhs`` override
    the size for scaled-down parity cases of the same shape."""
    if index == 0:
        n = n or 4096
        return Workload(0, "strip", strip(n), 64, 1e-6, np.array([math.pi / 6]), "c128")
    if index == 1:
        n = n or 65536
        return Workload(1, "parabola", parabola(n), 64, 1e-6, np.array([math.pi / 6]), "c64")
    if index == 2:
        n = n or (1 << 20)
        r = nrhs or 64
        return Workload(2, "spiral", archimedean_spiral(n), 64, 1e-6, uniform_angles(r), "c64")
    if index == 3:
        n = n or (1 << 18)
        w = Workload(3, "semicircle", semicircle(n), 64, 1e-6, np.array([math.pi / 6]), "c128")
        w.z = impedance(n, SEED_BASE + 3)
        return w
    if index == 4:
        n = n or (1 << 22)
        r = nrhs or 256
        return Workload(4, "multi", multi_curve(n), 64, 1e-6, uniform_angles(r), "c64")
    raise ValueError(f"no workload {index}")
