"""Parity against the FP64 oracle at the workloads' full sizes, in the launch
configurations the benchmark times.

- 100k convexes at 1297x840: the whole frame, forward and the L1 training
  gradient of every pixel.
- 1M convexes at 1920x1080: 5 % of the pixels, made of every pixel of the four
  longest tile lists (the multi-batch record pipeline, early termination and
  the long back-to-front recovery of T in the backward pass) plus a seeded
  uniform sample; forward and gradients per element.
- 500k convexes x 32 views of mixed resolution, batched, replayed from a
  captured hipGraph with the autotuner's tiling: sampled pixels of one view per
  resolution, forward and per-element gradients summed over those views.
- Serving: a 2M-convex 1920x1080 request served in a mixed batch, sampled
  pixels, plus the smaller requests of the same mix in full.
Bars: pixels 1e-4 absolute against the oracle's matched mode; gradients 1e-3
relative per tensor and per element, the element bar taken against at least
1e-2 of the tensor's rms and of the element's sum of |products| (the oracle's
magnitude: a sum that cancels is only good to float32 roundoffs of it), plus
the terms of the pairs whose skip / stop decision is within 1 % of its
threshold (either precision may take them).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_helpers import DECISION_TAU, grad_check, pixel_check, say  # noqa: E402
from paper_2411_14974_amd import scenes  # noqa: E402


@pytest.fixture(scope="module")
def R():
    from paper_2411_14974_amd.binding import Renderer
    r = Renderer(0)
    yield r
    r.close()


def dev(scene):
    from paper_2411_14974_amd.binding import DeviceScene
    return DeviceScene.from_scene(scene, "cuda:0")


def flat_pixels(sel, W):
    return np.stack([sel % W, sel // W], 1).astype(np.int32)


@pytest.mark.timeout(900)
def test_config2_full_frame(R):
    import oracle
    from paper_2411_14974_amd.binding import make_params
    scene, cam, target = scenes.config2()
    W, H = cam.width, cam.height
    say(f"[C2-frame] render N={scene.n} {W}x{H}")
    ds = dev(scene)
    rgb, st = R.forward(ds, cam, make_params(), want_state=True)
    dl = R.l1_loss_grad(rgb, torch.from_numpy(target).cuda())
    g = R.backward(st, dl)
    torch.cuda.synchronize()
    say("[C2-frame] oracle forward, whole frame")
    ref, _, _ = oracle.render(scene, cam, mode=oracle.MODE_MATCHED)
    pixel_check(rgb, ref, "C2-frame fwd")
    # the loss gradient the GPU computed is sign(C - target) / (3 W H)
    dl_np = dl.cpu().numpy()
    d = rgb.cpu().numpy() - target
    np.testing.assert_array_equal(dl_np, np.sign(d).astype(np.float32) / np.float32(d.size))
    say("[C2-frame] oracle backward, whole frame")
    gref = oracle.backward(scene, cam, dl_np.reshape(-1, 3), mode=oracle.MODE_MATCHED)
    scales = oracle.backward_magnitude(scene, cam, dl_np.reshape(-1, 3), tau=DECISION_TAU)
    grad_check(g, gref, "C2-frame bwd", scales)
    st.release()


@pytest.mark.timeout(900)
def test_config3_longest_lists_and_five_percent(R):
    import oracle
    from paper_2411_14974_amd.binding import make_params
    scene, cam, _ = scenes.config3()
    W, H = cam.width, cam.height
    say(f"[C3-5%] render N={scene.n} {W}x{H}")
    ds = dev(scene)
    rgb, st = R.forward(ds, cam, make_params(), want_state=True)
    torch.cuda.synchronize()
    ranges, ids = st.tile_lists()
    lens = ranges[:, 1] - ranges[:, 0]
    tx_n = (W + 15) // 16
    longest = np.argsort(-lens, kind="stable")[:4]
    say(f"[C3-5%] pairs {len(ids)}, longest lists {lens[longest].tolist()}, mean {lens.mean():.0f}")
    tile_pix = []
    for t in longest:
        tx, ty = int(t % tx_n), int(t // tx_n)
        for v in range(ty * 16, min(ty * 16 + 16, H)):
            for u in range(tx * 16, min(tx * 16 + 16, W)):
                tile_pix.append(v * W + u)
    rng = np.random.default_rng(31)
    want = (W * H) // 20
    rest = np.setdiff1d(rng.choice(W * H, want, replace=False), tile_pix)[: want - len(tile_pix)]
    sel = np.concatenate([np.array(tile_pix, np.int64), rest])
    assert len(np.unique(sel)) == len(sel) >= want
    pix = flat_pixels(sel, W)
    say(f"[C3-5%] oracle forward on {len(sel)} pixels")
    ref, _, nref = oracle.render(scene, cam, mode=oracle.MODE_MATCHED, pixels=pix)
    pixel_check(rgb, ref[: len(tile_pix)], "C3 longest tiles", sel=sel[: len(tile_pix)])
    pixel_check(rgb, ref, "C3 5%", sel=sel)
    say(f"[C3-5%] contributors per pixel in the longest tiles: max {int(nref[:len(tile_pix)].max())}")
    dl = np.zeros((H * W, 3), np.float32)
    dl[sel] = rng.normal(size=(len(sel), 3)).astype(np.float32)
    g = R.backward(st, torch.from_numpy(dl.reshape(H, W, 3)).cuda())
    torch.cuda.synchronize()
    say("[C3-5%] oracle backward")
    gref = oracle.backward(scene, cam, dl[sel], mode=oracle.MODE_MATCHED, pixels=pix)
    scales = oracle.backward_magnitude(scene, cam, dl[sel], pixels=pix, tau=DECISION_TAU)
    grad_check(g, gref, "C3 5%", scales)
    st.release()


@pytest.mark.timeout(900)
def test_config4_graph_autotuned_full_size(R):
    import oracle
    from paper_2411_14974_amd.binding import FLAG_AUTOTUNE, FLAG_GRAPH, make_params
    scene, cams, _ = scenes.config4()
    say(f"[C4] N={scene.n}, {len(cams)} views; autotune")
    ds = dev(scene)
    tune = R.autotune(ds, cams)
    say(f"[C4] tuning {tune}")
    p = make_params(flags=FLAG_GRAPH | FLAG_AUTOTUNE)
    outs, st = R.forward_batch(ds, cams, p, want_state=True)  # first call: eager, captures
    torch.cuda.synchronize()
    st.release()
    outs = [torch.full_like(o, -1.0) for o in outs]
    outs, st = R.forward_batch(ds, cams, p, want_state=True, outs=outs)  # replay
    assert R.batch_check(st) == 0
    rng = np.random.default_rng(41)
    picks = {}
    for v, c in enumerate(cams):
        picks.setdefault((c.width, c.height), v)
    assert len(picks) == 3
    dls = [torch.zeros_like(o) for o in outs]
    gref = mag = amb = None
    for (w, h), v in sorted(picks.items()):
        cam = cams[v]
        sel = rng.choice(w * h, 8000, replace=False)
        pix = flat_pixels(sel, w)
        say(f"[C4] view {v} {w}x{h}: oracle forward on {len(sel)} pixels")
        ref, _, _ = oracle.render(scene, cam, mode=oracle.MODE_MATCHED, pixels=pix)
        pixel_check(outs[v], ref, f"C4 view {v} {w}x{h}", sel=sel)
        d = np.zeros((h * w, 3), np.float32)
        d[sel] = rng.normal(size=(len(sel), 3)).astype(np.float32)
        dls[v].copy_(torch.from_numpy(d.reshape(h, w, 3)))
        say(f"[C4] view {v}: oracle backward")
        o = oracle.backward(scene, cam, d[sel], mode=oracle.MODE_MATCHED, pixels=pix)
        m, a = oracle.backward_magnitude(scene, cam, d[sel], pixels=pix, tau=DECISION_TAU)
        if gref is None:
            gref, mag, amb = o, m, a
        else:
            gref = {k: gref[k] + o[k] for k in o}
            mag = {k: mag[k] + m[k] for k in m}
            amb = {k: amb[k] + a[k] for k in a}
    g = R.backward_batch(st, dls)
    torch.cuda.synchronize()
    grad_check(g, gref, "C4 graph+autotune, 3 views", (mag, amb))
    st.release()


@pytest.mark.timeout(900)
def test_served_two_million_convexes_1080p(R):
    import oracle
    from paper_2411_14974_amd.binding import DeviceScene
    small = scenes.serve_scene(0)
    big = scenes.serve_scene(3)
    say(f"[C5] scenes {small.n} and {big.n} convexes")
    d_small, d_big = dev(small), dev(big)
    R.serve_start(workers=2, max_batch=4, start_paused=True)
    try:
        s0, s3 = R.scene_register(d_small), R.scene_register(d_big)
        rng = np.random.default_rng(51)
        reqs = []
        for sid, scene, (w, h) in ((s3, big, (1920, 1080)), (s3, big, (256, 256)), (s0, small, (960, 540)),
                                   (s0, small, (256, 256)), (s3, big, (960, 540))):
            cam = scenes.orbit_camera(rng, w, h)
            out = torch.full((h, w, 3), -1.0, device="cuda:0")
            reqs.append((scene, cam, out, R.serve_submit(sid, cam, out)))
        R.serve_resume()
        for *_, rid in reqs:
            R.serve_wait(rid)
        st = R.serve_stats()
        say(f"[C5] served: {st}")
        assert st["completed"] == len(reqs) and st["failed"] == 0
        torch.cuda.synchronize()
        for i, (scene, cam, out, _) in enumerate(reqs):
            w, h = cam.width, cam.height
            sel = np.arange(w * h) if w * h <= 65536 else rng.choice(w * h, 20000, replace=False)
            say(f"[C5] request {i}: N={scene.n} {w}x{h}, oracle on {len(sel)} pixels")
            ref, _, _ = oracle.render(scene, cam, mode=oracle.MODE_MATCHED, pixels=flat_pixels(sel, w))
            pixel_check(out, ref, f"C5 request {i} N={scene.n} {w}x{h}", sel=sel)
    finally:
        R.serve_stop()
