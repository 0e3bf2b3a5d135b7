"""GPU tests of the autotuner: it times every candidate (tile shape, fuse),
records the fastest, and automatic calls afterwards use the recorded
configuration with results identical bit for bit to the default one (and to
the FP64 oracle at relative L2 <= 1e-5); the table survives a save / clear /
load cycle; a batched plan built after ctv_batched_autotune uses its choice."""
import numpy as np
import pytest

import synth
from oracle import tv

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def ctv():
    import paper_2109_05496_amd as m
    return m


@pytest.fixture(autouse=True)
def clean_table():
    ctv().tune_cache_clear()
    yield
    ctv().tune_cache_clear()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def f32(t):
    return t.view(torch.float32)


@pytest.mark.parametrize("m,n,kind,K", [(200, 330, "1i", 30), (64, 64, "2a", 25), (130, 70, "1a", 9)])
def test_autotune_records_fastest_and_keeps_results(tmp_path, m, n, kind, K):
    rng = np.random.default_rng(11)
    _, b = synth.denoise_case(m, n, 12, 0.15, rng)
    mask = synth.square_mask(m, n, 0.7, rng)
    bt, mt = torch.as_tensor(b.astype(np.complex64)).cuda(), torch.as_tensor(mask).cuda()
    lam, alpha = 0.08, 0.4
    x_default = ctv().denoise(bt, lam, kind=kind, alpha=alpha, support=mt, iters=K, fuse=8, tile=(8, 8))
    assert ctv().tuned(m, n, kind=kind, alpha=alpha, iters=K) is None
    x_tune = torch.empty_like(bt)
    r = ctv().autotune(bt, lam, kind=kind, alpha=alpha, support=mt, iters=K, reps=2, out=x_tune)
    cands = r["candidates"]
    assert len(cands) >= 4
    best = r["best"]
    assert best["ms"] == min(c["ms"] for c in cands) and best in cands
    assert all(c["ms"] > 0 for c in cands)
    # every candidate computes the same x: the one left in out equals the default
    assert torch.equal(f32(x_tune), f32(x_default))
    got = ctv().tuned(m, n, kind=kind, alpha=alpha, iters=K)
    assert got == dict(fuse=best["fuse"], tile=best["tile"])
    T, _, w, rp = ctv().tiling(0, K, m, n, detail=True, kind=kind)
    assert (T, (w, rp)) == (min(best["fuse"], K), best["tile"])
    # an automatic call now runs the tuned configuration, same bits
    x_auto = ctv().denoise(bt, lam, kind=kind, alpha=alpha, support=mt, iters=K)
    torch.cuda.synchronize()
    assert torch.equal(f32(x_auto), f32(x_default))
    ref = tv.fgp(b.astype(np.complex64).astype(np.complex128), lam, K, kind, alpha, "modulus", mask)
    assert rel(x_auto.cpu().numpy().astype(np.complex128), ref) <= 1e-5
    # a different problem class (other K) is not affected
    assert ctv().tuned(m, n, kind=kind, alpha=alpha, iters=K + 1) is None
    # save / clear / load
    path = tmp_path / "tune.jsonl"
    ctv().tune_cache_save(path)
    ctv().tune_cache_clear()
    assert ctv().tuned(m, n, kind=kind, alpha=alpha, iters=K) is None
    ctv().tune_cache_load(path)
    assert ctv().tuned(m, n, kind=kind, alpha=alpha, iters=K) == got


def test_autotune_batch_of_images_and_prox_lookup():
    rng = np.random.default_rng(5)
    B, m, n, K = 3, 96, 160, 20
    bs = np.stack([synth.denoise_case(m, n, 8, 0.1, rng)[1] for _ in range(B)]).astype(np.complex64)
    bt = torch.as_tensor(bs).cuda()
    lams = [0.02, 0.05, 0.1]
    x_default = ctv().denoise(bt, lams, iters=K, fuse=8, tile=(8, 8))
    r = ctv().autotune(bt, lams, iters=K, reps=1)
    x_auto = ctv().denoise(bt, lams, iters=K)
    torch.cuda.synchronize()
    assert torch.equal(f32(x_auto), f32(x_default))
    assert ctv().tuned(m, n, batch=B, iters=K) == dict(fuse=r["best"]["fuse"], tile=r["best"]["tile"])
    assert ctv().tuned(m, n, batch=1, iters=K) is None


def test_batched_autotune_plan_uses_choice():
    rng = np.random.default_rng(3)
    specs = [(150, 90, "1i", 0.05, 24), (64, 200, "2a", 0.1, 17), (33, 47, "1a", 0.2, 9), (128, 128, "2i", 0.03, 24)]
    imgs, bs = [], []
    for mm, nn, kind, lam, K in specs:
        imgs.append(dict(m=mm, n=nn, lam=lam, kind=kind, alpha=0.3 if kind[0] == "2" else 0.5, iters=K))
        bs.append(synth.denoise_case(mm, nn, 6, 0.15, rng)[1].astype(np.complex64))
    plain_plan = ctv().BatchedPlan(imgs, fuse=8, tile=(8, 8))
    bp = plain_plan.pack(bs)
    x_ref = plain_plan.run(bp).clone()
    plain_plan.close()
    xt = torch.empty_like(bp)
    r = ctv().autotune_batched(imgs, bp, reps=1, out=xt)
    best = r["best"]
    assert best["ms"] == min(c["ms"] for c in r["candidates"])
    assert torch.equal(f32(xt), f32(x_ref))
    assert ctv().batched_tuned(imgs) == dict(fuse=best["fuse"], tile=best["tile"])
    assert ctv().batched_tuned(imgs[:3]) is None
    plan = ctv().BatchedPlan(imgs)
    assert plan.tiling == (best["fuse"], best["tile"][0], best["tile"][1])
    x = plan.run(bp)
    torch.cuda.synchronize()
    assert torch.equal(f32(x), f32(x_ref))
    plan.close()
    # a plan of other images keeps the default
    other = ctv().BatchedPlan(imgs[:3])
    assert other.tiling == (8, 8, 8)
    other.close()


def saved_table_entries():
    """(kind, fuse, tile) of the saved MI355X table's entries for the masked
    2048^2, K = 200 benchmark problem, read from the text of the table."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2109_05496_amd",
                        "tuning", "mi355x.jsonl")
    out = []
    for line in open(path):
        if not line.strip():
            continue
        e = json.loads(line)
        words = e["what"].split()
        if words[0] == "plain" and "m=2048" in words and "n=2048" in words and "K=200" in words:
            out.append((words[1], e["fuse"], (e["tile_waves"], e["tile_rows"])))
    return out


def test_benchmark_configuration_at_full_size_equals_default():
    """The masked 2048^2 four-kind workload in the launch configuration the
    benchmark runs (the saved table's entries) gives the same bits as the
    default configuration, which the corner-crop test pins to the oracle."""
    entries = saved_table_entries()
    assert sorted(k for k, _, _ in entries) == ["1a", "1i", "2a", "2i"]
    c = synth.config2(0)
    bt, mt = torch.as_tensor(c["b"]).cuda(), torch.as_tensor(c["mask"]).cuda()
    for kind, fuse, tile in entries:
        args = dict(kind=kind, alpha=c["alpha"], support=mt, iters=c["iters"])
        x_default = ctv().denoise(bt, c["lam"], fuse=8, tile=(8, 8), **args)
        x_bench = ctv().denoise(bt, c["lam"], fuse=fuse, tile=tile, **args)
        torch.cuda.synchronize()
        assert torch.equal(f32(x_bench), f32(x_default)), (kind, fuse, tile)


def test_benchmark_plan_at_full_size_equals_plain_calls():
    """The benchmark's step: the masked 2048^2 four-kind workload as one batched
    plan in the saved table's configuration (live tiles only). Every image
    equals the default plain call bit for bit, which the corner-crop test pins
    to the oracle."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2109_05496_amd",
                        "tuning", "mi355x.jsonl")
    c = synth.config2(0)
    m, n = c["b"].shape
    descs = [dict(m=m, n=n, lam=c["lam"], kind=k, alpha=c["alpha"], iters=c["iters"], has_support=True)
             for k in c["kinds"]]
    ctv().tune_cache_clear()
    ctv().tune_cache_load(path)
    try:
        assert ctv().batched_tuned(descs) is not None
        plan = ctv().BatchedPlan(descs)
        out = plan.unpack(plan.run(plan.pack([c["b"]] * 4), plan.pack_support([c["mask"]] * 4)))
        bt, mt = torch.as_tensor(c["b"]).cuda(), torch.as_tensor(c["mask"]).cuda()
        for i, kind in enumerate(c["kinds"]):
            ref = ctv().denoise(bt, c["lam"], kind=kind, alpha=c["alpha"], support=mt, iters=c["iters"], fuse=8,
                                tile=(8, 8))
            assert torch.equal(f32(out[i].reshape(m, n)), f32(ref)), kind
        plan.close()
    finally:
        ctv().tune_cache_clear()
