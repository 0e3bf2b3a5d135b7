"""GPU tests of the batched ragged path (one HIP-graph launch per call): each
image equals a plain ctv_denoise call bit for bit, and matches the FP64
oracle at relative L2 <= 1e-5."""
import numpy as np
import pytest

import synth
from _parity import ELEM_TOL, elem
from oracle import tv

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def ctv():
    import paper_2109_05496_amd as m
    return m


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def awkward_batch(seed=0):
    rng = np.random.default_rng(seed)
    specs = [(1, 1, "1i", 0.1, 10), (1, 70, "1a", 0.05, 23), (66, 1, "2i", 0.2, 17), (37, 53, "2a", 0.08, 30),
             (130, 150, "1i", 0.03, 41), (64, 64, "1a", 0.0, 20), (48, 90, "2i", 0.1, 0), (200, 77, "1i", 0.15, 1),
             (96, 140, "2a", 0.06, 33), (129, 129, "1a", 0.12, 8)]
    imgs, bs, masks = [], [], []
    for i, (m, n, kind, lam, K) in enumerate(specs):
        _, b = synth.denoise_case(m, n, 5, 0.15, rng)
        b = (b * 1.5).astype(np.complex64)
        has = i in (3, 4, 8)
        if has:
            masks.append(synth.square_mask(m, n, 0.6, rng))
        imgs.append(dict(m=m, n=n, lam=lam, kind=kind, alpha=0.3 if kind[0] == "2" else 0.5, iters=K,
                         has_support=has))
        bs.append(b)
    return imgs, bs, masks


def plain(b, d, mask):
    return ctv().denoise(torch.as_tensor(b).cuda(), d["lam"], kind=d["kind"], alpha=d["alpha"],
                         iters=d["iters"], support=None if mask is None else torch.as_tensor(mask).cuda())


def test_batched_equals_plain_bitwise_and_oracle():
    imgs, bs, masks = awkward_batch()
    plan = ctv().BatchedPlan(imgs)
    bp = plan.pack(bs)
    sp = plan.pack_support(masks)
    out1 = plan.unpack(plan.run(bp, sp))
    # a second call with fresh buffers exercises the graph-parameter update
    bp2 = bp.clone()
    out2 = plan.unpack(plan.run(bp2, sp.clone()))
    torch.cuda.synchronize()
    mit = iter(masks)
    for i, (d, b) in enumerate(zip(imgs, bs)):
        mask = next(mit) if d["has_support"] else None
        ref = plain(b, d, mask).cpu().numpy()
        x1, x2 = out1[i].cpu().numpy(), out2[i].cpu().numpy()
        assert np.array_equal(x1.view(np.uint32), ref.view(np.uint32)), i
        assert np.array_equal(x2.view(np.uint32), ref.view(np.uint32)), i
        xo = tv.fgp(b.astype(np.complex128), d["lam"], d["iters"], d["kind"], d["alpha"], "modulus", mask)
        assert rel(x1, xo) <= 1e-5, (i, rel(x1, xo))
        assert elem(x1, xo) <= ELEM_TOL, (i, elem(x1, xo))
    plan.close()


def test_batched_rejects_bad_descriptors():
    m = ctv()
    with pytest.raises(m.CtvError):
        m.BatchedPlan([dict(m=0, n=4, lam=0.1)])
    with pytest.raises(m.CtvError):
        m.BatchedPlan([dict(m=4, n=4, lam=-1.0)])
    with pytest.raises(m.CtvError):
        m.BatchedPlan([dict(m=4, n=4, lam=0.1, kind="2i", alpha=2.0)])


def test_config3_full_batch_matches_plain_calls():
    """The full ragged workload (256 images, 128..1024 per side, K = 150) in the
    launch configuration the benchmark times: every image equals its plain
    call bit for bit; the two smallest images also match the oracle."""
    imgs3 = synth.config3(0)
    descs = [dict(m=d["b"].shape[0], n=d["b"].shape[1], lam=d["lam"], kind=d["kind"], alpha=0.5,
                  iters=d["iters"]) for d in imgs3]
    plan = ctv().BatchedPlan(descs)
    bp = plan.pack([d["b"] for d in imgs3])
    out = plan.unpack(plan.run(bp))
    torch.cuda.synchronize()
    sizes = [d["b"].size for d in imgs3]
    for i, d in enumerate(imgs3):
        ref = ctv().denoise(torch.as_tensor(d["b"]).cuda(), d["lam"], kind=d["kind"], iters=d["iters"])
        assert torch.equal(out[i].view(torch.float32), ref.view(torch.float32)), i
    for i in np.argsort(sizes)[:2]:
        d = imgs3[i]
        xo = tv.fgp(d["b"].astype(np.complex128), d["lam"], d["iters"], d["kind"])
        assert rel(out[i].cpu().numpy(), xo) <= 1e-5, i
        assert elem(out[i].cpu().numpy(), xo) <= ELEM_TOL, i
    plan.close()


def test_batched_gradient_projection_method():
    imgs, bs, masks = awkward_batch(seed=3)
    plan = ctv().BatchedPlan(imgs, method="gp")
    out = plan.unpack(plan.run(plan.pack(bs), plan.pack_support(masks)))
    torch.cuda.synchronize()
    mit = iter(masks)
    for i, (d, b) in enumerate(zip(imgs, bs)):
        mask = next(mit) if d["has_support"] else None
        ref = ctv().denoise(torch.as_tensor(b).cuda(), d["lam"], kind=d["kind"], alpha=d["alpha"],
                            iters=d["iters"], support=None if mask is None else torch.as_tensor(mask).cuda(),
                            method="gp").cpu().numpy()
        x = out[i].cpu().numpy()
        assert np.array_equal(x.view(np.uint32), ref.view(np.uint32)), i
        xo = tv.fgp(b.astype(np.complex128), d["lam"], d["iters"], d["kind"], d["alpha"], "modulus", mask,
                    method="gp")
        assert rel(x, xo) <= 1e-5, (i, rel(x, xo))
        assert elem(x, xo) <= ELEM_TOL, (i, elem(x, xo))
    plan.close()


def test_packed_offsets_past_2_to_31_bytes():
    """A plan whose first image is 8192^2 (with a support, 2 GiB of dual state)
    and whose later images therefore start past 2^31 bytes into the packed
    state and past 2^28 elements into the packed inputs: every image equals
    the plain call bit for bit (the plain path is checked against the oracle
    at 8192^2 and 16384^2 on crops)."""
    rng = np.random.default_rng(7)
    c = synth.config2(0, size=8192, n_shapes=40)
    big_b = c["b"]
    big_mask = c["mask"]
    small = [(300, 500, "1a", 0.05, 12), (1000, 64, "2i", 0.1, 16), (65, 129, "1i", 0.08, 9)]
    imgs = [dict(m=8192, n=8192, lam=c["lam"], kind="1i", alpha=0.5, iters=16, has_support=True)]
    bs, masks = [big_b], [big_mask]
    for m, n, kind, lam, K in small:
        _, b = synth.denoise_case(m, n, 5, 0.15, rng)
        imgs.append(dict(m=m, n=n, lam=lam, kind=kind, alpha=0.3 if kind[0] == "2" else 0.5, iters=K,
                         has_support=False))
        bs.append((b * 1.5).astype(np.complex64))
    plan = ctv().BatchedPlan(imgs)
    out = plan.unpack(plan.run(plan.pack(bs), plan.pack_support(masks)))
    torch.cuda.synchronize()
    for i, (d, b) in enumerate(zip(imgs, bs)):
        ref = plain(b, d, big_mask if i == 0 else None)
        assert torch.equal(out[i].reshape(d["m"], d["n"]), ref), i
    plan.close()
