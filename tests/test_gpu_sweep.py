"""The row-sweep tile (tile_waves = -2): eight waves sweep down a 64-column
strip one iteration behind each other, with no vertical halo. It runs the same
per-pixel operators as the column-register tiles, so every result must equal
theirs bit for bit: all kinds and constraint sets, with and without a support,
every fusion depth it allows, segment heights that split the image into one or
several segments with ragged tails, resumed runs, checkpoints, the duality
gap, batched plans and the live-tile lists. One case is also checked against
the FP64 oracle."""
import numpy as np
import pytest

import synth
from _parity import ELEM_TOL, elem, rel
from oracle import tv

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

SWEEP = -2


def ctv():
    import paper_2109_05496_amd as m
    return m


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def case(shape, seed, scale=1.4):
    rng = np.random.default_rng(seed)
    _, b = synth.denoise_case(shape[0], shape[1], 8, 0.15, rng)
    return (b * scale).astype(np.complex64)


def bits(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("kind", tv.KINDS)
def test_sweep_equals_column_tile_bitwise(kind):
    rng = np.random.default_rng(3)
    for shape, seg in (((1, 1), 64), ((1, 67), 64), ((70, 1), 128), ((37, 53), 64), ((130, 150), 64),
                       ((300, 200), 128), ((517, 301), 256), ((260, 129), 64)):
        b = dev(case(shape, 10 + shape[0]))
        mask = dev(synth.square_mask(shape[0], shape[1], 0.6, rng))
        for constraint in ("modulus", "none"):
            for support in (None, mask):
                for K, fuse in ((23, 8), (17, 10), (9, 1), (12, 4), (31, 7)):
                    kw = dict(kind=kind, alpha=0.35, constraint=constraint, support=support, iters=K, fuse=fuse)
                    ref = ctv().denoise(b, 0.07, tile=(8, 8), **kw)
                    x = ctv().denoise(b, 0.07, tile=(SWEEP, seg), **kw)
                    assert np.array_equal(bits(x), bits(ref)), (kind, shape, seg, constraint, support is None, K, fuse)


def test_sweep_zero_iterations_and_zero_lambda():
    """K = 0 and lambda = 0 give x = P_C(b) through the sweep's output step alone."""
    rng = np.random.default_rng(9)
    b = dev(case((150, 97), 3, scale=1.8))
    mask = dev(synth.square_mask(150, 97, 0.5, rng))
    for lam, K in ((0.2, 0), (0.0, 13)):
        for support in (None, mask):
            ref = ctv().denoise(b, lam, iters=K, support=support, tile=(8, 8))
            x = ctv().denoise(b, lam, iters=K, support=support, tile=(SWEEP, 64))
            assert np.array_equal(bits(x), bits(ref)), (lam, K, support is None)


@pytest.mark.parametrize("kind", ["1i", "2a"])
def test_sweep_state_gap_resume_and_checkpoints(kind):
    b = dev(np.stack([case((211, 190), 5), case((211, 190), 6)]))
    lams = [0.05, 0.12]
    ref_x, ref_g, ref_st = ctv().denoise(b, lams, kind=kind, iters=29, gap=True, return_state=True, tile=(8, 8))
    x, g, st = ctv().denoise(b, lams, kind=kind, iters=29, gap=True, return_state=True, tile=(SWEEP, 64))
    assert np.array_equal(bits(x), bits(ref_x))
    assert np.array_equal(g.cpu().numpy().view(np.uint64), ref_g.cpu().numpy().view(np.uint64))
    assert np.array_equal(bits(st), bits(ref_st))
    # resume from the column tile's state with the sweep, and the other way round
    _, st1 = ctv().denoise(b, lams, kind=kind, iters=11, return_state=True, tile=(8, 8))
    x2 = ctv().denoise(b, lams, kind=kind, iters=18, state=st1, k0=11, tile=(SWEEP, 128))
    assert np.array_equal(bits(x2), bits(ref_x))
    # checkpoints every 10 (the state at 10 and 20 lands in caller slots)
    xc, saved = ctv().denoise(b, lams, kind=kind, iters=29, ckpt_every=10, tile=(SWEEP, 64))
    xr, saved_r = ctv().denoise(b, lams, kind=kind, iters=29, ckpt_every=10, tile=(8, 8))
    assert np.array_equal(bits(xc), bits(xr))
    assert np.array_equal(bits(saved), bits(saved_r))


def test_sweep_matches_oracle():
    c = synth.config2(0, size=320, n_shapes=30)
    b, mask = c["b"], c["mask"]
    for kind in ("1i", "2i"):
        x = ctv().denoise(dev(b), c["lam"], kind=kind, support=dev(mask), iters=40, tile=(SWEEP, 128))
        x = x.cpu().numpy()
        xo = tv.fgp(b.astype(np.complex128), c["lam"], 40, kind, 0.5, "modulus", mask)
        print("sweep", kind, "rel-L2", rel(x, xo), "elementwise", elem(x, xo))
        assert rel(x, xo) <= 1e-5 and elem(x, xo) <= ELEM_TOL


def test_sweep_batched_plan_equals_plain():
    rng = np.random.default_rng(8)
    specs = [(1, 1, "1i", 0.1, 10), (66, 1, "2i", 0.2, 17), (37, 53, "2a", 0.08, 30), (300, 150, "1i", 0.03, 41),
             (64, 64, "1a", 0.0, 20), (200, 77, "1i", 0.15, 1), (257, 190, "2a", 0.06, 33), (129, 129, "1a", 0.12, 8)]
    imgs, bs, masks = [], [], []
    for i, (m, n, kind, lam, K) in enumerate(specs):
        bs.append(case((m, n), 40 + i))
        has = i in (2, 3, 6)
        if has:
            masks.append(synth.square_mask(m, n, 0.6, rng))
        imgs.append(dict(m=m, n=n, lam=lam, kind=kind, alpha=0.3 if kind[0] == "2" else 0.5, iters=K,
                         has_support=has))
    for fuse in (8, 10, 3):
        plan = ctv().BatchedPlan(imgs, fuse=fuse, tile=(SWEEP, 64))
        assert plan.tiling == (fuse, SWEEP, 64)
        out = plan.unpack(plan.run(plan.pack(bs), plan.pack_support(masks)))
        torch.cuda.synchronize()
        mit = iter(masks)
        for i, (d, bb) in enumerate(zip(imgs, bs)):
            mk = next(mit) if d["has_support"] else None
            ref = ctv().denoise(dev(bb), d["lam"], kind=d["kind"], alpha=d["alpha"], iters=d["iters"], fuse=fuse,
                                support=None if mk is None else dev(mk), tile=(8, 8))
            assert np.array_equal(bits(out[i]), bits(ref)), (fuse, i)
        plan.close()


def test_sweep_live_tiles_equal_every_tile():
    """With a support and a cold start the sweep runs only its live tiles; a
    warm start from a zero state runs them all; both give the same bits."""
    c = synth.config2(0, size=700, n_shapes=60)
    b, mask = dev(c["b"]), dev(c["mask"])
    zero = torch.zeros((1, 2, 700, 700, 4), dtype=torch.float32, device="cuda")
    for kind in ("1a", "2i"):
        for seg in (64, 256):
            x = ctv().denoise(b, c["lam"], kind=kind, support=mask, iters=27, tile=(SWEEP, seg))
            xe = ctv().denoise(b, c["lam"], kind=kind, support=mask, iters=27, tile=(SWEEP, seg), state=zero, k0=0)
            assert np.array_equal(bits(x), bits(xe)), (kind, seg)
