"""The seeded generators are deterministic and produce the documented shapes."""
import numpy as np

import synth


def test_config1_deterministic_and_shaped():
    a, b = synth.config1(0), synth.config1(0)
    assert a["b"].dtype == np.complex64 and a["b"].shape == (64, 64)
    np.testing.assert_array_equal(a["b"], b["b"])
    amp = np.abs(a["truth"])
    assert amp.min() >= 0.2 - 1e-12 and amp.max() <= 1.0 + 1e-12


def test_square_mask_coverage():
    m = synth.square_mask(2048, 2048, 0.7, np.random.default_rng(0))
    assert m.dtype == np.uint8
    assert abs(m.mean() - 0.7) < 1e-3
    rows = np.where(m.any(1))[0]
    cols = np.where(m.any(0))[0]
    assert rows.size == cols.size == 1713 and m[rows[0]:rows[-1] + 1, cols[0]:cols[-1] + 1].all()


def test_config3_ragged():
    imgs = synth.config3(0, count=8)
    for d in imgs:
        H, W = d["b"].shape
        assert 128 <= H <= 1024 and 128 <= W <= 1024
        assert 0.01 <= d["lam"] <= 0.2 and d["kind"] in ("1i", "1a")
    assert len({d["b"].shape for d in imgs}) > 1


def test_noise_is_circular():
    z = synth.cn_noise((400, 400), 0.2, np.random.default_rng(1))
    assert abs(z.real.var() - 0.02) < 1e-3 and abs(z.imag.var() - 0.02) < 1e-3


def test_pr_object_and_poisson():
    x = synth.config5_object(seed=0, size=64, n_shapes=5, sigma_px=2.0)
    a, ph = np.abs(x), np.angle(x)
    assert a.min() >= 0.3 - 1e-12 and a.max() < 1.0
    assert ph.min() >= -1e-12 and ph.max() < 2.0
    y = synth.poisson_measure(np.full((50, 50), 2.0), 1000.0, np.random.default_rng(0))
    assert y.dtype == np.float32 and abs(y.mean() - 2.0) < 0.01


def test_phase_object_and_gaussian_noise():
    x = synth.phase_object(seed=3, size=96, n_shapes=8)
    assert x.shape == (96, 96)
    assert np.allclose(np.abs(x), 1.0)
    ph = np.angle(x)
    assert ph.min() >= -1e-12 and ph.max() < np.pi
    assert len(np.unique(np.round(ph, 12))) <= 9  # piecewise constant: background + 8 shapes at most
    assert np.array_equal(x, synth.phase_object(seed=3, size=96, n_shapes=8))
    rng = np.random.default_rng(0)
    I = np.full((200, 200), 2.0)
    y = synth.gaussian_measure(I, 0.1, rng)
    assert y.dtype == np.float32
    assert abs(float(y.mean()) - 2.0) < 0.01 and abs(float(y.std()) - 0.2) < 0.01
