"""Oracle pins: thin-lens circle of confusion, zone of focus (section 3.3,
eq. 6) and the aperture sampler used for the thin-lens rays (3.2.2)."""

import json
import math
import os

import numpy as np
import pytest

from paper_2210_06158_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def optics_coc(lens, width, z):
    """Blur diameter from the lens equation 1/f = 1/z + 1/v (binary64):
    a |v(z) - v(d)| / v(z) on the sensor, in pixels."""
    f, d, ws, N = (float(np.float32(x)) for x in (lens.focal, lens.focus, lens.sensor, lens.fnum))
    a = f / N
    vd = f * d / (d - f)
    if math.isinf(z):
        v = f
    else:
        v = f * z / (z - f)
    return a * abs(v - vd) / v * width / ws


def test_coc_matches_lens_equation(orc):
    rng = synth.SplitMix64(7)
    for fnum, d in ((1.4, 15.0), (2.0, 3.0), (8.0, 40.0), (1.0, 0.8)):
        lens = synth.Lens(fnum=fnum, focus=d)
        for z in np.concatenate([rng.uniform(50, 0.2, 200.0), [d, 1e6]]):
            got = orc.coc(lens, 1920, float(np.float32(z)))
            want = optics_coc(lens, 1920, float(np.float32(z)))
            assert got == pytest.approx(want, rel=2e-5, abs=1e-6), (fnum, d, z)


def test_coc_golden_small_workload(orc):
    g = json.load(open(os.path.join(GOLD, "coc_small.json")))
    lens = synth.Lens(**g["lens"])
    for case in g["cases"]:
        z = math.inf if case["z"] == "inf" else case["z"]
        assert orc.coc(lens, g["width"], z) == pytest.approx(case["coc_px"], rel=2e-5, abs=1e-7)


def test_coc_zero_at_focus_and_monotone(orc):
    lens = synth.Lens()
    assert orc.coc(lens, 256, lens.focus) == 0.0
    zs = np.linspace(0.3, lens.focus, 400)
    near = [orc.coc(lens, 256, float(z)) for z in zs]
    assert all(a >= b for a, b in zip(near, near[1:]))
    zs = np.linspace(lens.focus, 500.0, 400)
    far = [orc.coc(lens, 256, float(z)) for z in zs]
    assert all(a <= b for a, b in zip(far, far[1:]))


def eq6_bounds(lens, wi):
    """Eq. (6) written out in binary64."""
    f, d, ws = lens.focal, lens.focus, lens.sensor
    a = f / lens.fnum
    g = math.sqrt(2.0) * (d - f) * ws / wi
    lo = a * f * d / (a * f + g)
    hi = a * f * d / (a * f - g) if a * f > g else math.inf
    return lo, hi


@pytest.mark.parametrize("fnum,d,wi", [(1.4, 15.0, 256), (1.4, 15.0, 1920), (2.0, 3.0, 3840),
                                       (16.0, 40.0, 1920), (64.0, 15.0, 256)])
def test_zone_of_focus_eq6(orc, fnum, d, wi):
    lens = synth.Lens(fnum=fnum, focus=d)
    lo, hi = orc.zone(lens, wi)
    elo, ehi = eq6_bounds(lens, wi)
    assert lo == pytest.approx(elo, rel=1e-5)
    if math.isinf(ehi):
        assert math.isinf(hi)
    else:
        assert hi == pytest.approx(ehi, rel=1e-4)
        # a point at the far bound is one pixel diagonal across (3.3)
        assert orc.coc(lens, wi, hi) == pytest.approx(math.sqrt(2.0), rel=1e-4)
    assert orc.coc(lens, wi, lo) == pytest.approx(math.sqrt(2.0), rel=1e-4)
    # strictly inside the zone the CoC is below sqrt(2)
    mid = lo * 1.001 if math.isinf(hi) else 0.5 * (lo + hi)
    assert orc.coc(lens, wi, mid) < math.sqrt(2.0)


def _samples(orc, n, blades=0, rot=0.0):
    pts = np.array([orc.lens_sample(11, 3, q, k, blades, rot) for q in range(n // 64) for k in range(64)])
    return pts


def test_disc_sampler_moments(orc):
    p = _samples(orc, 64 * 1500)
    r2 = (p ** 2).sum(1)
    assert (r2 < 1.0).all()
    assert abs(p[:, 0].mean()) < 0.01 and abs(p[:, 1].mean()) < 0.01
    # uniform on the unit disc: E[r^2] = 1/2, P(r < 1/2) = 1/4
    assert r2.mean() == pytest.approx(0.5, abs=0.006)
    assert (r2 < 0.25).mean() == pytest.approx(0.25, abs=0.01)
    # samples are exact multiples of 2^-23 in [-1, 1)
    assert np.all(p * 2 ** 23 == np.round(p * 2 ** 23)) and p.min() >= -1.0 and p.max() < 1.0


def test_hexagon_sampler_inside_and_moment(orc):
    rot = 0.3
    p = _samples(orc, 64 * 1500, 6, rot)
    # inside test by the hexagon's own vertices (cross products), binary64
    verts = [(math.cos(rot + i * math.pi / 3), math.sin(rot + i * math.pi / 3)) for i in range(6)]
    for i in range(6):
        (x0, y0), (x1, y1) = verts[i], verts[(i + 1) % 6]
        cross = (x1 - x0) * (p[:, 1] - y0) - (y1 - y0) * (p[:, 0] - x0)
        assert (cross >= -1e-6).all()
    # regular hexagon of circumradius 1: E[r^2] = J / A = 5/12
    assert ((p ** 2).sum(1)).mean() == pytest.approx(5.0 / 12.0, abs=0.006)


def test_sampler_depends_on_every_counter(orc):
    base = orc.lens_sample(1, 2, 3, 4)
    for args in ((9, 2, 3, 4), (1, 9, 3, 4), (1, 2, 9, 4), (1, 2, 3, 9)):
        assert orc.lens_sample(*args) != base
