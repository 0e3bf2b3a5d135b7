"""Stream capture: ctv_denoise (per-step, dataflow and single-tile schedules,
with the duality gap), ctv_denoise_backward and pr_prox_grad with a fixed step
record into a HIP graph (torch.cuda.CUDAGraph) and every replay, with new
inputs copied in and eager library calls and synchronisations in between,
reproduces the eager call bit for bit."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def ctv():
    import paper_2109_05496_amd as m
    return m


def bits(t):
    return t.contiguous().view(torch.uint8)


def capture(fn):
    """Runs fn once on a side stream, then records it into a graph."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = fn()
    torch.cuda.synchronize()
    return g, out


def test_out_argument_is_returned_and_checked():
    b = torch.as_tensor(noisy(40, 70, 9)).cuda()
    out = torch.empty_like(b)
    assert ctv().denoise(b, 0.1, iters=5, out=out) is out
    with pytest.raises(ValueError):
        ctv().denoise(b, 0.1, iters=5, out=torch.empty((1, 40, 70), dtype=torch.complex64, device="cuda"))


def noisy(m, n, seed):
    rng = np.random.default_rng(seed)
    return (synth.denoise_case(m, n, 10, 0.15, rng)[1] * 1.3).astype(np.complex64)


@pytest.mark.parametrize("m,n,schedule,method", [(200, 300, "steps", "fgp"), (200, 300, "flow", "fgp"),
                                                 (64, 64, "auto", "fgp"), (130, 97, "steps", "gp")])
def test_denoise_graph_replays_match_eager(m, n, schedule, method):
    K, lam, kind = 27, 0.07, "2i"
    rng = np.random.default_rng(1)
    mask = torch.as_tensor(synth.square_mask(m, n, 0.7, rng)).cuda()
    b_static = torch.as_tensor(noisy(m, n, 100)).cuda()
    x_static = torch.empty_like(b_static)
    ws = torch.empty(ctv().workspace_size(m, n, 1, iters=K)[0], dtype=torch.uint8, device="cuda")

    def run():
        return ctv().denoise(b_static, lam, kind=kind, alpha=0.4, support=mask, iters=K, gap=True, out=x_static,
                             workspace=ws, method=method, schedule=schedule)

    g, (x_cap, gap_cap) = capture(run)
    assert x_cap.data_ptr() == x_static.data_ptr() and x_cap.shape == x_static.shape
    for rep in range(3):
        new = torch.as_tensor(noisy(m, n, rep)).cuda()
        b_static.copy_(new)
        g.replay()
        torch.cuda.synchronize()
        x_eager, gap_eager = ctv().denoise(new, lam, kind=kind, alpha=0.4, support=mask, iters=K, gap=True,
                                           method=method, schedule=schedule)
        torch.cuda.synchronize()
        assert torch.equal(bits(x_cap), bits(x_eager)), f"replay {rep}"
        assert torch.equal(bits(gap_cap), bits(gap_eager)), f"replay {rep}"


def test_backward_graph_replays_match_eager():
    B, m, n, K, c, lam = 2, 96, 130, 23, 5, 0.05
    b = torch.as_tensor(np.stack([noisy(m, n, 7 + i) for i in range(B)])).cuda()
    _, saved = ctv().denoise(b, lam, iters=K, ckpt_every=c)
    gx_static = torch.empty_like(b)
    gx_static.copy_(torch.as_tensor(np.stack([noisy(m, n, 50 + i) for i in range(B)])).cuda())

    def run():
        return ctv().denoise_backward(b, lam, gx_static, saved, iters=K, ckpt_every=c)

    g, (gb_cap, gl_cap) = capture(run)
    for rep in range(3):
        new = torch.as_tensor(np.stack([noisy(m, n, 200 + 10 * rep + i) for i in range(B)])).cuda()
        gx_static.copy_(new)
        g.replay()
        torch.cuda.synchronize()
        gb, gl = ctv().denoise_backward(b, lam, new, saved, iters=K, ckpt_every=c)
        torch.cuda.synchronize()
        assert torch.equal(bits(gb_cap), bits(gb)), f"replay {rep}"
        assert torch.equal(bits(gl_cap), bits(gl)), f"replay {rep}"


def test_phase_retrieval_fixed_step_graph_replays_match_eager():
    m = 128
    P = synth.PR_DEFAULTS
    truth = synth.config5_object(seed=3, size=m, n_shapes=8)
    fields = ctv().pr_forward(torch.as_tensor(truth.astype(np.complex64)).cuda(), P["distances"], P["wavelength"],
                              P["pixel"])
    inten = (fields.abs() ** 2).cpu().numpy().astype(np.float64)

    def measure(seed):
        rng = np.random.default_rng(seed)
        return torch.as_tensor(np.stack([synth.poisson_measure(I, P["photons"], rng) for I in inten])).cuda()

    y_static = measure(0)

    def run():
        return ctv().phase_retrieval(y_static, P["distances"], P["wavelength"], P["pixel"], tau=0.01, gamma=0.25,
                                     outer=6, inner=10, loss=True)

    g, (x_cap, loss_cap) = capture(run)
    for rep in range(3):
        new = measure(1 + rep)
        y_static.copy_(new)
        g.replay()
        torch.cuda.synchronize()
        x, loss = ctv().phase_retrieval(new, P["distances"], P["wavelength"], P["pixel"], tau=0.01, gamma=0.25,
                                        outer=6, inner=10, loss=True)
        torch.cuda.synchronize()
        assert torch.equal(bits(x_cap), bits(x)), f"replay {rep}"
        assert torch.equal(bits(loss_cap), bits(loss)), f"replay {rep}"


def test_autotune_refuses_stream_capture():
    """The autotuner synchronises the host, so it returns an error (before any
    device work) when its stream is being captured; the capture itself stays
    usable."""
    b = torch.as_tensor(noisy(64, 96, 3)).cuda()
    counter = torch.zeros(1, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        counter.add_(1.0)
        with pytest.raises(ctv().CtvError) as err:
            ctv().autotune(b, 0.1, iters=5, reps=1)
    assert "capture" in str(err.value)
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    assert float(counter.cpu()) == 3.0
