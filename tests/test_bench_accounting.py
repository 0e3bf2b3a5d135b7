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
