"""Repeated runs give the same bits: the forward solver (per-step and dataflow
schedules, with the duality gap), a batched plan, the backward pass (whose
lambda gradient is a reduction) and phase retrieval. A race on LDS or on the
cross-tile state would show up here as run-to-run differences."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

REPEATS = 5


def ctv():
    import paper_2109_05496_amd as m
    return m


def bits(t):
    return t.contiguous().view(torch.uint8).clone()


def noisy(m, n, seed, batch=None):
    rng = np.random.default_rng(seed)
    if batch is None:
        return torch.as_tensor((synth.denoise_case(m, n, 12, 0.15, rng)[1] * 1.3).astype(np.complex64)).cuda()
    return torch.as_tensor(np.stack([(synth.denoise_case(m, n, 12, 0.15, rng)[1] * 1.3).astype(np.complex64)
                                     for _ in range(batch)])).cuda()


def same_every_time(fn):
    first = [bits(t) for t in fn()]
    for rep in range(REPEATS - 1):
        again = [bits(t) for t in fn()]
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(first, again)):
            assert torch.equal(a, b), (rep, i)


@pytest.mark.parametrize("kind", ["1i", "1a", "2i", "2a"])
@pytest.mark.parametrize("schedule", ["steps", "flow"])
def test_denoise_and_gap_repeat_bitwise(kind, schedule):
    b = noisy(300, 257, 4)
    mask = torch.as_tensor(synth.square_mask(300, 257, 0.7, np.random.default_rng(2))).cuda()
    same_every_time(lambda: ctv().denoise(b, 0.06, kind=kind, alpha=0.35, support=mask, iters=37, gap=True,
                                          schedule=schedule))


def test_batched_plan_repeats_bitwise():
    rng = np.random.default_rng(8)
    imgs, bs = [], []
    for i, (m, n) in enumerate([(150, 90), (64, 200), (33, 47), (300, 128)]):
        kind = ["1i", "1a", "2i", "2a"][i]
        imgs.append(dict(m=m, n=n, lam=0.03 + 0.02 * i, kind=kind, alpha=0.4, iters=20 + 7 * i))
        bs.append((synth.denoise_case(m, n, 6, 0.15, rng)[1]).astype(np.complex64))
    plan = ctv().BatchedPlan(imgs)
    bp = plan.pack(bs)
    same_every_time(lambda: [plan.run(bp)])
    plan.close()


def test_backward_repeats_bitwise():
    b = noisy(96, 130, 6, batch=3)
    _, saved = ctv().denoise(b, 0.05, iters=23, ckpt_every=5)
    gx = noisy(96, 130, 7, batch=3)
    same_every_time(lambda: ctv().denoise_backward(b, 0.05, gx, saved, iters=23, ckpt_every=5))


@pytest.mark.parametrize("size,outer", [(128, 5), (1024, 2)])
def test_phase_retrieval_repeats_bitwise(size, outer):
    """Also at 1024^2, where the gradient runs the round-trip and
    accumulate-inverse passes with one wave per line and four distances
    side by side, and the iterative-projection method."""
    P = synth.PR_DEFAULTS
    truth = synth.config5_object(seed=1, size=size, n_shapes=8)
    f = ctv().pr_forward(torch.as_tensor(truth.astype(np.complex64)).cuda(), P["distances"], P["wavelength"],
                         P["pixel"])
    rng = np.random.default_rng(3)
    y = torch.as_tensor(np.stack([synth.poisson_measure(I, P["photons"], rng)
                                  for I in (f.abs() ** 2).cpu().numpy().astype(np.float64)])).cuda()
    same_every_time(lambda: ctv().phase_retrieval(y, P["distances"], P["wavelength"], P["pixel"], tau=0.01,
                                                  gamma=0.25, outer=outer, inner=10, loss=True))
    same_every_time(lambda: ctv().phase_retrieval_ip(y, P["distances"], P["wavelength"], P["pixel"], iters=outer,
                                                     loss=True))
