"""The benchmark's own arithmetic, on the CPU: the accuracy judge's SSIM
against closed forms and a window-by-window restatement, and the traffic
summary reader (calibration scales, source fingerprint)."""

import hashlib
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

torch = pytest.importorskip("torch")

W709 = np.array([0.2126, 0.7152, 0.0722])
C1, C2 = 0.01 ** 2, 0.03 ** 2


def ssim_windows(a, b):
    """Mean SSIM of the luma of two images, one 11 x 11 Gaussian window
    (sigma 1.5) at a time, with weighted means, variances and covariance
    (Wang et al. 2004, eq. 13 with its constants for a unit range)."""
    la, lb = a @ W709, b @ W709
    x = np.arange(11) - 5.0
    g = np.exp(-x * x / (2 * 1.5 ** 2))
    w = np.outer(g, g) / np.outer(g, g).sum()
    H, Wd = la.shape
    vals = []
    for i in range(H - 10):
        for j in range(Wd - 10):
            pa, pb = la[i:i + 11, j:j + 11], lb[i:i + 11, j:j + 11]
            ma, mb = (w * pa).sum(), (w * pb).sum()
            va, vb = (w * (pa - ma) ** 2).sum(), (w * (pb - mb) ** 2).sum()
            cab = (w * (pa - ma) * (pb - mb)).sum()
            vals.append((2 * ma * mb + C1) * (2 * cab + C2) / ((ma * ma + mb * mb + C1) * (va + vb + C2)))
    return float(np.mean(vals))


def test_ssim_of_an_image_with_itself_is_one():
    rng = np.random.default_rng(3)
    a = torch.from_numpy(rng.uniform(0, 1, (24, 30, 3)))
    assert bench.ssim_luma(a, a) == pytest.approx(1.0, abs=1e-12)


def test_ssim_of_constant_images_is_the_luminance_term():
    # no variance anywhere: SSIM reduces to (2 mu_a mu_b + C1) / (mu_a^2 + mu_b^2 + C1)
    a = torch.full((16, 16, 3), 0.25, dtype=torch.float64)
    b = torch.full((16, 16, 3), 0.75, dtype=torch.float64)
    want = (2 * 0.25 * 0.75 + C1) / (0.25 ** 2 + 0.75 ** 2 + C1)
    assert bench.ssim_luma(a, b) == pytest.approx(want, rel=1e-9)


def test_ssim_of_an_inverted_pattern_is_negative():
    # b = 1 - a on every channel: the structure term flips sign
    rng = np.random.default_rng(4)
    a = rng.uniform(0, 1, (20, 20, 1)).repeat(3, axis=2)
    s = bench.ssim_luma(torch.from_numpy(a), torch.from_numpy(1.0 - a))
    assert s < -0.5


@pytest.mark.parametrize("seed", [5, 6])
def test_ssim_matches_the_window_by_window_definition(seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0, 1, (19, 23, 3))
    b = np.clip(a + rng.normal(0, 0.08, a.shape), 0, 1)
    got = bench.ssim_luma(torch.from_numpy(a), torch.from_numpy(b))
    assert got == pytest.approx(ssim_windows(a, b), abs=1e-10)


def write_traffic(tmp_path, sources, sha=None, **kv):
    h = hashlib.sha256()
    for p in sources:
        h.update(open(p, "rb").read())
    lines = ["# header line with = sign that is a comment", f"source_sha256={sha or h.hexdigest()}"]
    lines += [f"{k}={v}" for k, v in kv.items()]
    path = tmp_path / "traffic.txt"
    path.write_text("\n".join(lines) + "\n")
    return str(path)


def test_measured_traffic_scales_both_counters(tmp_path, monkeypatch):
    srcs = []
    for name, text in (("a.hip", "kernel a"), ("b.hip", "kernel b")):
        p = tmp_path / name
        p.write_text(text)
        srcs.append(str(p))
    path = write_traffic(tmp_path, srcs, fetch_kib_per_launch=1000.0, write_kib_per_launch=300.0,
                         fetch_scale=2.0, write_scale=1.0, tcc_hit_per_launch=900, tcc_miss_per_launch=100)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", path)
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", srcs)
    mt = bench.measured_traffic()
    assert mt["hbm_bytes"] == (1000 * 2 + 300) * 1024
    assert mt["tcc_hit"] == 900 and mt["tcc_miss"] == 100
    l2 = bench.l2_figure(mt, 2.0)
    assert l2["requests_per_launch"] == 1000 and l2["hit_rate"] == 0.9
    assert l2["grequests_per_s"] == pytest.approx(1000 / 2e-3 / 1e9, abs=0.01)


def test_measured_traffic_is_none_once_a_source_changes(tmp_path, monkeypatch):
    p = tmp_path / "k.hip"
    p.write_text("v1")
    path = write_traffic(tmp_path, [str(p)], fetch_kib_per_launch=1.0, write_kib_per_launch=1.0,
                         fetch_scale=1.0, write_scale=1.0)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", path)
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", [str(p)])
    assert bench.measured_traffic() is not None
    p.write_text("v2")
    assert bench.measured_traffic() is None


def test_committed_traffic_summary_parses():
    kv = dict(l.split("=", 1) for l in open(bench.TRAFFIC_FILE).read().split("\n") if "=" in l and not l.startswith("#"))
    for k in ("source_sha256", "fetch_kib_per_launch", "write_kib_per_launch", "fetch_scale", "write_scale"):
        assert k in kv
    assert all(math.isfinite(float(kv[k])) for k in ("fetch_kib_per_launch", "write_kib_per_launch"))


def test_tuner_keeps_the_incumbent_within_its_margin():
    from paper_2210_06158_amd import tune
    times = {16: 10.0, 24: 9.95, 32: 10.4}
    assert tune.pick(times) == 24                              # the fastest
    assert tune.pick(times, incumbent=16, margin=0.01) == 16   # 0.5 % slower: kept
    assert tune.pick(times, incumbent=32, margin=0.01) == 24   # 4.5 % slower: replaced
    assert tune.pick(times, incumbent=40, margin=0.01) == 24   # not a candidate
    assert tune.pick({1: 5.0}, incumbent=1, margin=0.0) == 1
