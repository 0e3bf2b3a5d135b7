"""Tiles outside the support. With a support mask and a cold start, ctv_denoise
runs only the tiles whose output holds a pixel where the dual can move (in the
support, or with a support pixel below or to the right; that the dual stays
exactly zero everywhere else is pinned on the oracle in test_oracle_fgp.py),
from a live-tile list built once per tiling. Results must be bitwise those of
running every tile, which a warm start from an all-zero state does (the lists
need a cold start). Workspaces are filled with NaN bytes first, so any stale
state that a skipped tile left behind would show."""
import numpy as np
import pytest

import synth
from oracle import tv

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

TOL = 1e-5


def ctv():
    import paper_2109_05496_amd as m
    return m


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def bits(t):
    return t.cpu().numpy().view(np.uint32)


def sparse_mask(m, n):
    """A block well inside, one pixel in the last row and column, and a strip
    along the right border: dead tiles in the interior and at every border."""
    mk = np.zeros((m, n), np.uint8)
    mk[m // 3:m // 3 + m // 5, n // 4:n // 4 + n // 6] = 1
    mk[m - 1, n - 1] = 1
    mk[5:m // 2, n - 3:] = 1
    return mk


def nan_workspace(m, n, B, kind, iters, fuse):
    ws_bytes, _ = ctv().workspace_size(m, n, B, kind, 0.5, "modulus", iters, fuse, 0, "fgp")
    return torch.full((ws_bytes,), 0xFF, dtype=torch.uint8, device="cuda")


def zero_state(B, m, n):
    return torch.zeros((B, 2, m, n, 4), dtype=torch.float32, device="cuda")


SHAPES = [(8, 8), (8, 4), (4, 8), (12, 4), (16, 4), (16, 8)]


@pytest.mark.parametrize("kind", tv.KINDS)
def test_skipping_is_bitwise_invisible(kind):
    m, n = 300, 420
    rng = np.random.default_rng(41)
    _, b = synth.denoise_case(m, n, 12, 0.15, rng)
    mask = dev(sparse_mask(m, n))
    bt = dev(b)
    for tile in SHAPES:
        for fuse, iters in ((3, 20), (8, 37), (9, 30)):
            kw = dict(kind=kind, support=mask, iters=iters, fuse=fuse, tile=tile)
            ws = nan_workspace(m, n, 1, kind, iters, fuse)
            x, g, st = ctv().denoise(bt, 0.07, gap=True, return_state=True, workspace=ws, **kw)
            xd, gd, std = ctv().denoise(bt, 0.07, gap=True, return_state=True, state=zero_state(1, m, n),
                                        k0=0, **kw)
            assert np.array_equal(bits(x), bits(xd)), (tile, fuse)
            assert np.array_equal(bits(st), bits(std)), (tile, fuse)
            assert torch.equal(g, gd), (tile, fuse)
            # the third and later launches reuse both ping-pong buffers; the
            # gap variant also keeps the final state in one of them
            xg = ctv().denoise(bt, 0.07, gap=True, workspace=ws, **kw)[0]
            assert np.array_equal(bits(xg), bits(x)), (tile, fuse)
            # x alone, from a fresh NaN-filled workspace
            xr = ctv().denoise(bt, 0.07, workspace=nan_workspace(m, n, 1, kind, iters, fuse), **kw)
            assert np.array_equal(bits(xr), bits(x)), (tile, fuse)


def test_skipping_matches_oracle_and_reused_workspace():
    """A workspace reused from a call with another support, a batch sharing the
    support, and the oracle at the stated tolerance."""
    m, n, K = 200, 260, 30
    rng = np.random.default_rng(42)
    bs = np.stack([synth.denoise_case(m, n, 10, 0.15, rng)[1] for _ in range(3)])
    mk = sparse_mask(m, n)
    ws = nan_workspace(m, n, 3, "2i", K, 0)
    full = dev(np.ones((m, n), np.uint8))
    ctv().denoise(dev(bs), [0.05, 0.08, 0.12], kind="2i", support=full, iters=K, workspace=ws)
    x = ctv().denoise(dev(bs), [0.05, 0.08, 0.12], kind="2i", support=dev(mk), iters=K, workspace=ws)
    x = x.cpu().numpy()
    for i, lam in enumerate((0.05, 0.08, 0.12)):
        xo = tv.fgp(bs[i].astype(np.complex128), lam, K, "2i", 0.5, "modulus", mk)
        err = np.linalg.norm(x[i] - xo) / np.linalg.norm(xo)
        assert err <= TOL, (i, err)
        assert np.all(x[i][mk == 0] == 0)


@pytest.mark.parametrize("kind", ["1i", "2a"])
def test_checkpoints_with_skipping_equal_resumed_states(kind):
    """Checkpoint slots are fresh buffers: dead tiles store their zeros there.
    Slot s holds the state after (s + 1) * c iterations, bitwise as a plain run
    returns it."""
    m, n, K, c = 180, 150, 30, 10
    rng = np.random.default_rng(43)
    _, b = synth.denoise_case(m, n, 10, 0.15, rng)
    mk = sparse_mask(m, n)
    bt, mt = dev(b), dev(mk)
    x, saved = ctv().denoise(bt, 0.06, kind=kind, support=mt, iters=K, ckpt_every=c)
    slot = saved.view(-1, 1, 2, m, n, 4)
    for s in range(slot.shape[0]):
        _, st = ctv().denoise(bt, 0.06, kind=kind, support=mt, iters=(s + 1) * c, return_state=True)
        assert np.array_equal(bits(slot[s]), bits(st)), s
    xn = ctv().denoise(bt, 0.06, kind=kind, support=mt, iters=K)
    assert np.array_equal(bits(x), bits(xn))


def test_tilings_chunks_and_single_launch():
    """K = 50 with T = 8 runs launches of 8 and 7 iterations and an x launch
    (three tilings, three lists); K = 5 is one launch that writes x; 33 images
    are two chunks of the batch, each with its own lists. The duality gap and
    the returned state match too."""
    m, n = 150, 230
    rng = np.random.default_rng(44)
    mk = dev(sparse_mask(m, n))
    for B, iters in ((1, 50), (1, 5), (33, 12)):
        bs = np.stack([synth.denoise_case(m, n, 6, 0.15, rng)[1] for _ in range(B)])
        bt = dev(bs)
        lams = list(np.linspace(0.04, 0.12, B))
        ws = nan_workspace(m, n, B, "1a", iters, 8)
        x, g = ctv().denoise(bt, lams, kind="1a", support=mk, iters=iters, fuse=8, workspace=ws, gap=True)
        xd, gd, std = ctv().denoise(bt, lams, kind="1a", support=mk, iters=iters, fuse=8,
                                    state=zero_state(B, m, n), k0=0, gap=True, return_state=True)
        assert np.array_equal(bits(x), bits(xd)), (B, iters)
        assert torch.equal(g, gd), (B, iters)
        xr = ctv().denoise(bt, lams, kind="1a", support=mk, iters=iters, fuse=8,
                           workspace=nan_workspace(m, n, B, "1a", iters, 8))
        assert np.array_equal(bits(xr), bits(xd)), (B, iters)
        xs, st = ctv().denoise(bt, lams, kind="1a", support=mk, iters=iters, fuse=8, workspace=ws,
                               return_state=True)
        assert np.array_equal(bits(xs), bits(xd)), (B, iters)
        assert np.array_equal(bits(st), bits(std)), (B, iters)


def test_support_of_one_pixel_and_of_nothing():
    """All tiles but one (or all) skipped: x is zero outside, the one pixel's
    neighbourhood matches the oracle."""
    m, n, K = 130, 190, 25
    rng = np.random.default_rng(45)
    _, b = synth.denoise_case(m, n, 6, 0.15, rng)
    one = np.zeros((m, n), np.uint8)
    one[77, 101] = 1
    for mask in (np.zeros((m, n), np.uint8), one):
        ws = nan_workspace(m, n, 1, "2i", K, 0)
        x = ctv().denoise(dev(b), 0.1, kind="2i", support=dev(mask), iters=K, workspace=ws).cpu().numpy()
        xo = tv.fgp(b.astype(np.complex128), 0.1, K, "2i", 0.5, "modulus", mask)
        assert np.all(x[mask == 0] == 0)
        assert np.allclose(x, xo, rtol=0, atol=1e-6)


def test_batched_plan_skips_dead_tiles_bitwise():
    """A batched plan runs only the live tiles of its images with a support
    (scan and list nodes ahead of the steps): every image equals the plain call
    that runs every tile, for ragged sizes and iteration counts, lambda = 0 and
    K = 0 images with a support, empty and full supports, images without one,
    and a NaN-filled workspace; a second run with new buffers patches the scan
    node."""
    rng = np.random.default_rng(46)
    specs = [(300, 420, "1i", 0.07, 37, "sparse"), (150, 230, "2a", 0.1, 12, "sparse"), (90, 70, "1a", 0.05, 20, None),
             (200, 260, "2i", 0.0, 15, "sparse"), (130, 190, "1i", 0.08, 0, "sparse"), (64, 64, "1a", 0.06, 9, "sparse"),
             (80, 120, "2i", 0.09, 14, "empty"), (100, 100, "1a", 0.05, 21, "full")]
    imgs, bs, masks = [], [], []
    for m, n, kind, lam, K, sup in specs:
        _, b = synth.denoise_case(m, n, 6, 0.15, rng)
        bs.append(b)
        imgs.append(dict(m=m, n=n, lam=lam, kind=kind, alpha=0.5, iters=K, has_support=sup is not None))
        if sup == "sparse":
            masks.append(sparse_mask(m, n))
        elif sup is not None:
            masks.append((np.ones if sup == "full" else np.zeros)((m, n), np.uint8))
    plan = ctv().BatchedPlan(imgs)
    bp, sp = plan.pack(bs), plan.pack_support(masks)
    plan._ws = torch.full((max(plan.ws_bytes, 1),), 0xFF, dtype=torch.uint8, device="cuda")
    out1 = plan.unpack(plan.run(bp, sp))
    out2 = plan.unpack(plan.run(bp.clone(), sp.clone()))
    mit = iter(masks)
    for i, (d, b) in enumerate(zip(imgs, bs)):
        mk = dev(next(mit)) if d["has_support"] else None
        m, n = d["m"], d["n"]
        ref = ctv().denoise(dev(b), d["lam"], kind=d["kind"], iters=d["iters"], support=mk,
                            state=zero_state(1, m, n) if d["iters"] and d["lam"] else None, k0=0)
        assert np.array_equal(bits(out1[i]), bits(ref)), i
        assert np.array_equal(bits(out2[i]), bits(ref)), i
    plan.close()


def blob_mask(m, n, rng):
    """A few random rectangles and single pixels (possibly none) on an empty
    support: every kind of live/dead tile neighbourhood."""
    mk = np.zeros((m, n), np.uint8)
    for _ in range(int(rng.integers(0, 4))):
        j0, k0 = int(rng.integers(0, m)), int(rng.integers(0, n))
        mk[j0:j0 + int(rng.integers(1, max(2, m // 3))), k0:k0 + int(rng.integers(1, max(2, n // 3)))] = 1
    for _ in range(int(rng.integers(0, 3))):
        mk[int(rng.integers(0, m)), int(rng.integers(0, n))] = 1
    return mk


def test_random_supports_plain_and_batched():
    """Twenty seeded random problems (sizes 1..300 per side, random supports,
    kinds, tile shapes, fusion depths and K): plain calls equal their every-tile
    runs, and one batched plan of all of them equals the plain calls."""
    rng = np.random.default_rng(47)
    shapes = [(8, 8), (8, 4), (4, 8), (12, 4), (16, 4), (16, 8)]
    imgs, bs, masks, outs = [], [], [], []
    for case in range(20):
        m, n = int(rng.integers(1, 301)), int(rng.integers(1, 301))
        kind = str(rng.choice(["1i", "1a", "2i", "2a"]))
        K = int(rng.integers(1, 30))
        fuse = int(rng.integers(1, 10))
        tile = shapes[int(rng.integers(0, len(shapes)))]
        b = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))).astype(np.complex64)
        mk = blob_mask(m, n, rng)
        bt, mt = dev(b), dev(mk)
        x = ctv().denoise(bt, 0.1, kind=kind, support=mt, iters=K, fuse=fuse, tile=tile,
                          workspace=nan_workspace(m, n, 1, kind, K, fuse))
        xd = ctv().denoise(bt, 0.1, kind=kind, support=mt, iters=K, fuse=fuse, tile=tile,
                           state=zero_state(1, m, n), k0=0)
        assert np.array_equal(bits(x), bits(xd)), (case, m, n, kind, K, fuse, tile)
        imgs.append(dict(m=m, n=n, lam=0.1, kind=kind, alpha=0.5, iters=K, has_support=True))
        bs.append(b)
        masks.append(mk)
        outs.append(x)
    plan = ctv().BatchedPlan(imgs)
    got = plan.unpack(plan.run(plan.pack(bs), plan.pack_support(masks)))
    for i, x in enumerate(outs):
        ref = ctv().denoise(dev(bs[i]), 0.1, kind=imgs[i]["kind"], support=dev(masks[i]), iters=imgs[i]["iters"])
        assert np.array_equal(bits(got[i]), bits(ref)), i
    plan.close()


@pytest.mark.parametrize("kind,ckpt", [("1i", 10), ("2a", 3), ("1a", 23)])
def test_backward_with_sparse_support_matches_oracle(kind, ckpt):
    """The reverse steps of ctv_denoise_backward run only the live tiles of the
    adjoint's tiling (the adjoint state stays zero where the dual does): a
    two-image batch with a sparse support against the oracle's reverse pass
    (relative L2 <= 1e-4, the adjoint bar), zero gradient outside the support,
    for three checkpoint spacings (reverse-step halos 6, 4 and 6)."""
    from oracle import adjoint as oadj
    m, n, K = 150, 230, 23
    rng = np.random.default_rng(48)
    mk = sparse_mask(m, n)
    bs = np.stack([synth.denoise_case(m, n, 8, 0.15, rng)[1] * 1.3 for _ in range(2)]).astype(np.complex64)
    xbar = (rng.standard_normal((2, m, n)) + 1j * rng.standard_normal((2, m, n))).astype(np.complex64)
    lams = [0.06, 0.11]
    bt, mt = dev(bs), dev(mk)
    x, saved = ctv().denoise(bt, lams, kind=kind, support=mt, iters=K, ckpt_every=ckpt)
    gb, gl = ctv().denoise_backward(bt, lams, dev(xbar), saved, kind=kind, support=mt, iters=K, ckpt_every=ckpt)
    gb, gl = gb.cpu().numpy(), gl.cpu().numpy()
    for i in range(2):
        _, gbo, glo = oadj.fgp_vjp(bs[i].astype(np.complex128), lams[i], K, xbar[i].astype(np.complex128), kind,
                                   0.5, "modulus", mk)
        err = np.linalg.norm(gb[i] - gbo) / np.linalg.norm(gbo)
        assert err <= 1e-4, (i, err)
        assert abs(gl[i] - glo) <= 1e-4 * max(1.0, abs(glo)), (i, gl[i], glo)
        assert np.all(gb[i][mk == 0] == 0)
