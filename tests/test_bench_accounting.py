"""Host-side accounting of bench.py (no GPU): the count of computed pixels that
the roofline uses follows the live-tile rule pixel by pixel, and the
multi-GPU request is refused."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def brute_live_tile_px(mask, halo, rows):
    m, n = mask.shape
    OW, OH = 64 - 2 * halo, rows - 2 * halo
    live_tiles = tiles = px = 0
    for ty in range(-(-m // OH)):
        for tx in range(-(-n // OW)):
            tiles += 1
            live = False
            cnt = 0
            for j in range(ty * OH, min(m, ty * OH + OH)):
                for k in range(tx * OW, min(n, tx * OW + OW)):
                    cnt += 1
                    near = mask[j, k] or (j + 1 < m and mask[j + 1, k]) or (k + 1 < n and mask[j, k + 1])
                    live = live or bool(near)
            if live:
                live_tiles += 1
                px += cnt
    return live_tiles, tiles, px


@pytest.mark.parametrize("seed", range(6))
def test_live_tile_px_matches_the_pixel_rule(seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(1, 140)), int(rng.integers(1, 140))
    mask = np.zeros((m, n), np.uint8)
    for _ in range(int(rng.integers(0, 4))):
        j0, k0 = int(rng.integers(0, m)), int(rng.integers(0, n))
        mask[j0:j0 + int(rng.integers(1, m + 1)), k0:k0 + int(rng.integers(1, n + 1))] = 1
    halo = int(rng.integers(1, 9))
    rows = int(rng.choice([32, 64]))
    assert bench.live_tile_px(mask, halo, rows) == brute_live_tile_px(mask, halo, rows)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _summary(path, doc):
    import json
    with open(path, "w") as f:
        f.write("# summary\n\n```json\n" + json.dumps(doc) + "\n```\n")


def test_profile_figures_per_unit_and_source_gate(tmp_path, monkeypatch):
    """The secondary roofline blocks read the committed rocprofv3 summaries:
    launches per unit are normalised by the marker kernel, the measured rate is
    traffic over the profiled duration, and a summary taken on other sources
    (hash mismatch) is ignored."""
    from paper_2109_05496_amd import prof_summary as ps
    g = ps.GROUPS["pr"]
    good = {"group": "pr", "sources": list(g["sources"]), "source_sha256": ps.source_hash(g["sources"])}
    (tmp_path / "profiles").mkdir()
    stats = dict(good, kernels={"void ctv::(anonymous namespace)::fft_acc_inverse_kernel<1024, true>(a)":
                                {"calls": 300, "avg_us": 20.0},
                                "void ctv::fgp_col_kernel<0, 1, false, 8, 4, false>(b)": {"calls": 900, "avg_us": 25.0},
                                "void ctv::(anonymous namespace)::fft_line_kernel<1024, 1, false>(c)":
                                {"calls": 300, "avg_us": 10.0}})
    pmc = dict(good, kernels={"void ctv::(anonymous namespace)::fft_acc_inverse_kernel<1024, true>(a)":
                              {"traffic_bytes": 80_000_000, "valu_issue_frac": 0.4},
                              "void ctv::fgp_col_kernel<0, 1, false, 8, 4, false>(b)":
                              {"traffic_bytes": 60_000_000, "valu_issue_frac": 0.5}})
    _summary(tmp_path / "profiles" / "s.md", stats)
    _summary(tmp_path / "profiles" / "p.md", pmc)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    figs = bench.profile_figures(("s.md", "p.md"), "fft_acc_inverse_kernel", ("fft_", "fgp_"))
    acc = figs["void ctv::(anonymous namespace)::fft_acc_inverse_kernel<1024, true>(a)"]
    fgp = figs["void ctv::fgp_col_kernel<0, 1, false, 8, 4, false>(b)"]
    line = figs["void ctv::(anonymous namespace)::fft_line_kernel<1024, 1, false>(c)"]
    assert acc["launches_per_unit"] == 1.0 and fgp["launches_per_unit"] == 3.0
    assert acc["hbm"]["achieved"] == pytest.approx(80e6 / 20e-6 / 1e9, rel=1e-3)
    assert acc["hbm"]["frac"] == pytest.approx(80e6 / 20e-6 / 1e9 / bench.HBM_PEAK_GBS, rel=1e-3)
    assert line["traffic_bytes"] is None and "hbm" not in line
    is_fft = lambda k: "fft_" in k  # noqa: E731
    assert bench._per_unit(figs, is_fft, "avg_us") == pytest.approx(30.0)
    assert bench._per_unit(figs, lambda k: True, "avg_us") == pytest.approx(105.0)
    assert bench._per_unit(figs, is_fft, "traffic_bytes") is None  # a kernel without counters
    assert bench._per_unit(figs, lambda k: "fgp_" in k, "traffic_bytes") == pytest.approx(180e6)
    stale = dict(stats, source_sha256="0" * 64)
    _summary(tmp_path / "profiles" / "s.md", stale)
    assert bench.profile_figures(("s.md", "p.md"), "fft_acc_inverse_kernel", ("fft_",)) is None


def test_committed_profiles_were_taken_on_the_committed_sources():
    """Every summary under profiles/ that carries a JSON block names its kernel
    group and the SHA-256 of that group's sources; it must be the hash of the
    sources in the tree, or bench.py would ignore the summary (and its numbers
    would describe other code)."""
    from paper_2109_05496_amd import prof_summary as ps
    prof = os.path.join(ROOT, "profiles")
    checked = 0
    for name in sorted(os.listdir(prof)):
        text = open(os.path.join(prof, name)).read()
        if "```json" not in text:
            continue
        doc = ps.load_summary(os.path.join(prof, name))
        assert doc is not None, f"{name}: taken on other sources than the ones in the tree"
        assert doc["group"] in ps.GROUPS
        checked += 1
    assert checked >= 8
