"""One training step of the rasterizer captured in one graph.

A batched render with a pair capacity never reads back to the host, and the
backward only launches kernels, so both can be recorded into one HIP graph
together with the caller's own loss: here a batched render of three views of
different sizes, the gradient of an L2 loss to seeded target images
(elementwise torch operations), and gs_render_backward.  The graph is replayed
several times, with eager work, synchronisations and a change of the targets
between the replays; every replay must give the images of the eager step bit
for bit and its gradients to float-atomic rounding (the backward sums each
Gaussian's per-tile terms with atomics, in no fixed order).
"""
import sys

import numpy as np
import pytest

import scenes

pytestmark = [pytest.mark.gpu]

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def l2_grads(outs, targets):
    """dL/d(image) of L = sum over views of mean((image - target)^2)."""
    return [(o["image"] - t) * (2.0 / t.numel()) for o, t in zip(outs, targets)]


def test_forward_loss_backward_in_one_captured_graph():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C2", n=20_000, seed=81)
    dev = gs.scene_to_device(sc)
    cams = [scenes.default_camera(160, 96), scenes.look_at_camera([1.5, -0.4, -2.4], 128, 128),
            scenes.look_at_camera([-2.0, 0.3, -2.0], 96, 200)]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    targets = [torch.rand((3, c["height"], c["width"]), device="cuda", generator=gen) for c in cams]

    ref = gs.Renderer(0)
    r = gs.Renderer(0)
    try:
        ref.render_batched(dev, cams)
        cap = int(ref.list_info()["num_pairs"] * 1.5) + 4096

        def eager_step():
            outs = ref.render_batched(dev, cams, pair_capacity=cap)
            grads = ref.backward(dev, l2_grads(outs, targets))
            torch.cuda.synchronize()
            return ([o["image"].cpu().numpy().view(np.uint32).copy() for o in outs],
                    {k: v.cpu().numpy() for k, v in grads.items()})

        # one eager step sizes every buffer of r's context; the capture then
        # allocates nothing on the device outside torch's graph pool
        outs = r.render_batched(dev, cams, pair_capacity=cap)
        r.backward(dev, l2_grads(outs, targets))
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            g_outs = r.render_batched(dev, cams, pair_capacity=cap)
            g_grads = r.backward(dev, l2_grads(g_outs, targets))
        torch.cuda.synchronize()
        for rep in range(4):
            if rep == 2:
                for t in targets:
                    t.mul_(0.5).add_(0.25)   # a new target, read by the next replays
            graph.replay()
            torch.cuda.synchronize()
            got_img = [o["image"].cpu().numpy().view(np.uint32).copy() for o in g_outs]
            got = {k: v.cpu().numpy() for k, v in g_grads.items()}
            want_img, want = eager_step()   # eager work between the replays
            for v in range(len(cams)):
                assert np.array_equal(got_img[v], want_img[v]), f"replay {rep} view {v}: image"
            errs = {}
            for k in GROUPS:
                w = want[k].astype(np.float64)
                d = got[k].astype(np.float64) - w
                nrm = float(np.linalg.norm(w))
                assert nrm > 0, k
                errs[k] = float(np.linalg.norm(d)) / nrm
                assert np.all(np.isfinite(got[k])), k
            say(f"[train graph] replay {rep}: " + " ".join(f"{k}={e:.1e}" for k, e in errs.items()))
            for k, e in errs.items():
                assert e < 1e-5, (rep, k, e)
    finally:
        r.close()
        ref.close()
