"""Seeded input generators: equal-arc-length nodes at 10 segments per
wavelength on the synthetic open curves, disjoint multi-curve layouts."""
import math

import mpmath as mp
import numpy as np

from paper_1901_11371_amd import inputs


def _seglen(c):
    return np.concatenate([np.linalg.norm(np.diff(c.xy[c.node_off[i]:c.node_off[i + 1]], axis=0), axis=1)
                           for i in range(c.ncurves)])


def test_curves_have_ten_segments_per_wavelength():
    for c in (inputs.strip(512), inputs.parabola(512), inputs.archimedean_spiral(512),
              inputs.semicircle(512), inputs.multi_curve(512)):
        assert c.n_segments == 512
        L = _seglen(c)
        assert np.all(np.abs(L - 0.1) < 1e-4), c.name   # chords of 0.1-long arcs


def test_spiral_and_parabola_arc_constants():
    # arc length of r = a theta over [pi, 6 pi] is a * integral sqrt(1 + t^2)
    unit = float(mp.quad(lambda t: mp.sqrt(1 + t * t), [mp.pi, 6 * mp.pi]))
    c = inputs.archimedean_spiral(1 << 12)
    assert abs(c.meta["a"] * unit - 409.6) < 1e-9
    # parabola y = 0.3 x^2 / Lp over [-Lp/2, Lp/2]: arc = Lp * integral_{-1/2}^{1/2} sqrt(1 + (0.6 u)^2) du
    g = float(mp.quad(lambda u: mp.sqrt(1 + (0.6 * u) ** 2), [-0.5, 0.5]))
    p = inputs.parabola(1 << 12)
    assert abs(p.meta["Lp"] * g - 409.6) < 1e-9


def test_multi_curve_disjoint_and_seeded():
    a = inputs.multi_curve(4096)
    b = inputs.multi_curve(4096)
    assert np.array_equal(a.xy, b.xy)
    assert a.ncurves == 8 and a.n_segments == 4096
    pts = [a.xy[a.node_off[i]:a.node_off[i + 1]] for i in range(8)]
    for i in range(8):
        for j in range(i + 1, 8):
            d = np.min(np.linalg.norm(pts[i][::4, None, :] - pts[j][None, ::4, :], axis=2))
            assert d > 1.0


def test_plane_wave_unit_amplitude():
    c = inputs.semicircle(256)
    b = inputs.plane_wave_rhs(c, inputs.uniform_angles(4))
    assert b.shape == (4, 256) and np.allclose(np.abs(b), 1)


def test_arc_families():
    for ang in (math.pi / 4, math.pi, 1.9 * math.pi):
        c = inputs.arc_with_angle(1024, ang)
        assert c.n_segments == 1024
        assert np.all(np.abs(_seglen(c) - 0.1) < 1e-4)
        # endpoints subtend the requested angle at the centre (on the y axis)
        r = c.meta["radius"]
        p0, p1 = c.xy[0], c.xy[-1]
        cy = p0[1] - r * math.sin(math.pi / 2 - ang / 2)
        a0 = math.atan2(p0[1] - cy, p0[0])
        a1 = math.atan2(p1[1] - cy, p1[0])
        assert abs(((a1 - a0) % (2 * math.pi)) - ang) < 1e-9
    a = inputs.arc_array(2048, 4, gap=2.0)
    assert a.ncurves == 4 and a.n_segments == 2048
    assert np.all(np.abs(_seglen(a) - 0.1) < 1e-4)
    # left to right, separated by the gap
    for k in range(3):
        end = a.xy[a.node_off[k + 1] - 1]
        start = a.xy[a.node_off[k + 1]]
        assert abs(np.linalg.norm(start - end) - 2.0) < 1e-9 and start[0] > end[0]
