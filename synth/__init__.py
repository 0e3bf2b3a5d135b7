"""Seeded synthetic inputs for the CTV-FGP denoiser and phase retrieval.

These stand in for the paper's test images (a phase-only "cameraman" image and
other standard test images), which are not available: piecewise-constant complex
images built from random disks and rectangles, complex Gaussian noise, square
support masks, ragged batches, and a smoothed random object for phase retrieval.

This module holds no arithmetic of the method (no differences, projections,
propagation or FGP step). It is shared by the tests, the benchmark and the
oracle-side checks only as a source of inputs. Every function takes an explicit
seed or ``numpy.random.Generator``; the draw order is fixed and documented so the
inputs are reproducible on any machine.
"""
import math

import numpy as np

__all__ = [
    "piecewise_complex", "cn_noise", "square_mask", "denoise_case", "config1",
    "config2", "config3", "config4", "config5_object", "poisson_measure",
    "PR_DEFAULTS", "PR_PAPER_SIM", "phase_object", "gaussian_measure",
]


def piecewise_complex(H, W, n_shapes, rng, amp=(0.2, 1.0), phase=(-math.pi, math.pi)):
    """Piecewise-constant complex image.

    Draw order: background amplitude, background phase; then per shape:
    kind (disk if U<0.5), centre row, centre column, size draw(s), amplitude,
    phase. Later shapes overwrite earlier ones. Disk radius is
    U[0.03, 0.2] * min(H, W); a rectangle has half-height U[0.03, 0.2] * H and
    half-width U[0.03, 0.2] * W.
    """
    a0 = rng.uniform(*amp)
    p0 = rng.uniform(*phase)
    img = np.full((H, W), a0 * np.exp(1j * p0), dtype=np.complex128)

    def box(c, half, size):
        # index range holding every pixel within `half` of c, one pixel of margin
        return max(0, int(math.floor(c - half)) - 1), min(size, int(math.ceil(c + half)) + 2)

    for _ in range(n_shapes):
        is_disk = rng.uniform() < 0.5
        cj = rng.uniform(0, H)
        ck = rng.uniform(0, W)
        if is_disk:
            rad = rng.uniform(0.03, 0.2) * min(H, W)
            (j0, j1), (k0, k1) = box(cj, rad, H), box(ck, rad, W)
            jj = np.arange(j0, j1)[:, None]
            kk = np.arange(k0, k1)[None, :]
            sel = (jj - cj) ** 2 + (kk - ck) ** 2 <= rad * rad
        else:
            hh = rng.uniform(0.03, 0.2) * H
            hw = rng.uniform(0.03, 0.2) * W
            (j0, j1), (k0, k1) = box(cj, hh, H), box(ck, hw, W)
            jj = np.arange(j0, j1)[:, None]
            kk = np.arange(k0, k1)[None, :]
            sel = (np.abs(jj - cj) <= hh) & (np.abs(kk - ck) <= hw)
        a = rng.uniform(*amp)
        p = rng.uniform(*phase)
        img[j0:j1, k0:k1][sel] = a * np.exp(1j * p)
    return img


def cn_noise(shape, sigma, rng):
    """Circular complex Gaussian CN(0, sigma^2): real and imaginary parts are
    independent N(0, sigma^2 / 2) (real part drawn first)."""
    s = sigma / math.sqrt(2.0)
    re = rng.normal(0.0, s, size=shape)
    im = rng.normal(0.0, s, size=shape)
    return re + 1j * im


def square_mask(H, W, frac, rng):
    """One axis-aligned square of side round(sqrt(frac*H*W)) (clipped to the
    image) at a uniformly drawn top-left corner; uint8 0/1."""
    side = int(round(math.sqrt(frac * H * W)))
    sh, sw = min(side, H), min(side, W)
    j0 = int(rng.integers(0, H - sh + 1))
    k0 = int(rng.integers(0, W - sw + 1))
    m = np.zeros((H, W), dtype=np.uint8)
    m[j0:j0 + sh, k0:k0 + sw] = 1
    return m


def denoise_case(H, W, n_shapes, sigma, rng):
    """(truth complex128, b complex64) with b = truth + CN(0, sigma^2), rounded
    once to complex64. Tests give the oracle the exact upcast of that b."""
    truth = piecewise_complex(H, W, n_shapes, rng)
    b = (truth + cn_noise((H, W), sigma, rng)).astype(np.complex64)
    return truth, b


def config1(seed=0):
    """Single 64 x 64 image, 6 shapes, sigma 0.1; type-1 isotropic, lambda 0.05,
    |x| <= 1, 100 iterations."""
    rng = np.random.default_rng(seed)
    truth, b = denoise_case(64, 64, 6, 0.1, rng)
    return dict(truth=truth, b=b, lam=0.05, kind="1i", alpha=0.5,
                constraint="modulus", mask=None, iters=100)


def config2(seed=0, size=2048, n_shapes=200):
    """size x size image, 200 shapes, sigma 0.15, lambda 0.08, |x| <= 1 with a
    square support mask covering 70 % of the pixels, 200 iterations, all four
    TV kinds (alpha = 1/2)."""
    rng = np.random.default_rng(seed)
    truth, b = denoise_case(size, size, n_shapes, 0.15, rng)
    mask = square_mask(size, size, 0.7, rng)
    return dict(truth=truth, b=b, lam=0.08, kinds=("1i", "1a", "2i", "2a"), alpha=0.5,
                constraint="modulus", mask=mask, iters=200)


def config3(seed=0, count=256, lo=128, hi=1024, iters=150):
    """Ragged batch: per image, height then width ~ U{lo..hi}, then
    lambda = exp(U[ln 0.01, ln 0.2]), then kind 1i/1a with probability 1/2,
    then the image itself (20 shapes, sigma 0.15). |x| <= 1, no mask."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        H = int(rng.integers(lo, hi + 1))
        W = int(rng.integers(lo, hi + 1))
        lam = float(np.exp(rng.uniform(np.log(0.01), np.log(0.2))))
        kind = "1i" if rng.uniform() < 0.5 else "1a"
        truth, b = denoise_case(H, W, 20, 0.15, rng)
        out.append(dict(truth=truth, b=b, lam=lam, kind=kind, alpha=0.5,
                        constraint="modulus", mask=None, iters=iters))
    return out


def config4(seed=0, batch=16, size=512):
    """Batch of equally sized images for the differentiable denoiser: 20 shapes,
    sigma 0.1, type-1 isotropic, lambda 0.05, 50 iterations, checkpoints every 10."""
    rng = np.random.default_rng(seed)
    truths, bs = [], []
    for _ in range(batch):
        t, b = denoise_case(size, size, 20, 0.1, rng)
        truths.append(t)
        bs.append(b)
    return dict(truth=np.stack(truths), b=np.stack(bs), lam=0.05, kind="1i", alpha=0.5,
                constraint="modulus", mask=None, iters=50, ckpt_every=10)


def _smooth_field(H, W, n_shapes, rng, sigma_px):
    from scipy.ndimage import gaussian_filter
    f = np.zeros((H, W))
    jj = np.arange(H)[:, None]
    kk = np.arange(W)[None, :]
    for _ in range(n_shapes):
        is_disk = rng.uniform() < 0.5
        cj = rng.uniform(0, H)
        ck = rng.uniform(0, W)
        if is_disk:
            rad = rng.uniform(0.03, 0.2) * min(H, W)
            sel = (jj - cj) ** 2 + (kk - ck) ** 2 <= rad * rad
        else:
            hh = rng.uniform(0.03, 0.2) * H
            hw = rng.uniform(0.03, 0.2) * W
            sel = (np.abs(jj - cj) <= hh) & (np.abs(kk - ck) <= hw)
        f[sel] = rng.uniform()
    if sigma_px > 0:
        f = gaussian_filter(f, sigma_px, mode="wrap")
    f = f - f.min()
    top = f.max()
    return f / (top * (1 + 1e-12)) if top > 0 else f


PR_DEFAULTS = dict(wavelength=532e-9, pixel=4e-6, distances=(1.0e-3, 1.5e-3, 2.0e-3, 2.5e-3),
                   photons=1000.0, outer=100, inner=20, tau=0.01, gamma=0.25,
                   kind="1i", alpha=0.5, constraint="modulus")


def config5_object(seed=0, size=1024, n_shapes=40, sigma_px=4.0):
    """Phase-retrieval object: amplitude 0.3 + 0.7 f_a and phase 2 f_p (rad),
    with f_a then f_p independent piecewise-constant random fields of n_shapes
    shapes, Gaussian-smoothed (sigma_px, periodic) and normalised to [0, 1)."""
    rng = np.random.default_rng(seed)
    fa = _smooth_field(size, size, n_shapes, rng, sigma_px)
    fp = _smooth_field(size, size, n_shapes, rng, sigma_px)
    return (0.3 + 0.7 * fa) * np.exp(1j * 2.0 * fp)


# The simulated experiment of Section VI-A: a 256 x 256 pure phase object with
# its phase in [0, pi), pixel 5 um, wavelength 500 nm, one distance of 5 mm,
# 10 % Gaussian noise on the intensity, type-I anisotropic TV, 10 FGP
# iterations per prox, all methods from the back-propagated field. The paper
# does not state tau; 0.01 here, with a sweep beside it.
PR_PAPER_SIM = dict(wavelength=500e-9, pixel=5e-6, distances=(5e-3,), noise=0.10, size=256, outer=100,
                    inner=10, tau=0.01, gamma=1.0, kind="1a", alpha=0.5)


def phase_object(seed=0, size=256, n_shapes=30):
    """Pure phase object exp(i pi f) (the stand-in for the paper's phase-only
    test images): f a piecewise-constant random field of n_shapes shapes
    (drawn as for config5_object, no smoothing, sharp edges) normalised to
    [0, 1), so the phase lies in [0, pi)."""
    rng = np.random.default_rng(seed)
    f = _smooth_field(size, size, n_shapes, rng, 0.0)
    return np.exp(1j * math.pi * f)


def gaussian_measure(intensity, rel_sigma, rng):
    """Intensity with additive white Gaussian noise whose standard deviation is
    rel_sigma times the mean intensity (the reading of "10 % Gaussian noise");
    float32, not clipped (the square root of the data clips at 0)."""
    intensity = np.asarray(intensity, dtype=np.float64)
    noise = rng.standard_normal(intensity.shape) * (rel_sigma * float(intensity.mean()))
    return (intensity + noise).astype(np.float32)


def poisson_measure(intensity, photons, rng):
    """Poisson counts at ``photons`` mean per pixel, rescaled back to the
    intensity's units: y = Poisson(photons * I / mean(I)) * mean(I) / photons."""
    intensity = np.asarray(intensity, dtype=np.float64)
    mu = float(intensity.mean())
    counts = rng.poisson(photons * intensity / mu)
    return (counts * (mu / photons)).astype(np.float32)
