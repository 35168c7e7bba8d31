"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: hull index sequences and depth keys bit-exact; per-tile lists hold every
convex the oracle finds with alpha >= eps_alpha in the tile, in depth order;
pixels within 1e-4 absolute of the oracle's matched mode; gradients (the same
dL/dC fed to both) within 1e-3 relative per tensor (L2) and per element
(floor 1e-2 rms).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2411_14974_amd import scenes  # noqa: E402
from paper_2411_14974_amd.scenes import Camera, Scene  # noqa: E402

PIX_TOL = 1e-4
GRAD_TOL = 1e-3
NAMES = ("points", "delta", "sigma", "opacity", "sh")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    from paper_2411_14974_amd.binding import Renderer
    r = Renderer(0)
    yield r
    r.close()


def dev(scene):
    from paper_2411_14974_amd.binding import DeviceScene
    return DeviceScene.from_scene(scene, "cuda:0")


def render_gpu(R, scene, cam, want_state=False, **kw):
    from paper_2411_14974_amd.binding import make_params
    ds = dev(scene)
    rgb, st = R.forward(ds, cam, make_params(**kw), want_state=want_state)
    torch.cuda.synchronize()
    return ds, rgb, st


def grad_check(g_gpu, g_ref, label):
    worst = {}
    for k in NAMES:
        a = g_gpu[k].detach().cpu().numpy().astype(np.float64).ravel()
        b = np.asarray(g_ref[k], np.float64).ravel()
        nb = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / max(nb, 1e-300)
        rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
        elem = np.abs(a - b) / np.maximum(np.abs(b), 1e-2 * rms + 1e-300)
        worst[k] = (float(rel), float(elem.max()) if b.size else 0.0)
    say(f"[{label}] grad rel-L2 / worst element: " + ", ".join(f"{k} {v[0]:.1e}/{v[1]:.1e}" for k, v in worst.items()))
    for k, (rel, el) in worst.items():
        assert rel <= GRAD_TOL, (label, k, rel)
        assert el <= GRAD_TOL, (label, k, el)


# ------------------------------------------------------------ preprocess ----

STATUS_MAP = {0: 0, 1: 1, 2: 2, 3: 0}  # GPU "faint" (opacity <= eps) is visible to the oracle


def check_preprocess(R, scene, cam, label):
    import oracle
    g = R.debug_preprocess(dev(scene), cam)
    o = oracle.preprocess(scene, cam)
    degenerate = 0
    ntiles_x = (cam.width + 15) // 16
    for i in range(scene.n):
        a, b = g[i], o[i]
        if b.status & 256:
            degenerate += 1
            continue
        assert STATUS_MAP[a.status] == (b.status & 0xFF), (label, i, a.status, b.status)
        if a.status == 1:
            continue
        assert a.T == b.T, (label, i)
        assert list(a.hull)[:a.T] == list(b.hull)[:b.T], (label, i)
        if a.status in (0, 3):
            assert a.depth_key == b.key, (label, i, hex(a.depth_key), hex(b.key))
            for j in range(a.T):
                assert abs(a.A[j] - b.nx[j]) < 1e-12 and abs(a.B[j] - b.ny[j]) < 1e-12, (label, i, j)
                assert abs(a.C[j] - b.off[j]) < 1e-9 * (1 + abs(b.off[j])), (label, i, j)
            assert abs(a.d - b.d) <= 1e-12 * b.d and abs(a.delta_p - b.dp) <= 1e-12 * b.dp
            assert abs(a.sigma_p - b.sp) <= 1e-12 * b.sp
            np.testing.assert_allclose(list(a.rgb), list(b.rgb), atol=2e-6)
            assert a.clampmask == b.clampmask or np.min(np.abs(list(b.rgb))) < 1e-6
        if a.status == 0:
            # the oracle's alpha >= eps region must lie inside the GPU's tile rectangle
            x0, y0, x1, y1 = b.rect
            u0, u1 = max(0, int(np.ceil(x0 - 0.5))), min(cam.width - 1, int(np.floor(x1 - 0.5)))
            v0, v1 = max(0, int(np.ceil(y0 - 0.5))), min(cam.height - 1, int(np.floor(y1 - 0.5)))
            if u0 <= u1 and v0 <= v1:
                tx0, ty0, tx1, ty1 = list(a.tile_rect)
                assert tx0 <= u0 // 16 and u1 // 16 <= tx1 and ty0 <= v0 // 16 and v1 // 16 <= ty1, (label, i)
    say(f"[{label}] preprocess parity over {scene.n} convexes, {degenerate} degenerate excluded")
    assert degenerate <= max(1, scene.n // 10000)


def test_preprocess_parity_config1(R):
    scene, cam = scenes.config1()
    check_preprocess(R, scene, cam, "C1")


def test_preprocess_parity_config2_subset(R):
    scene, cam, _ = scenes.config2(n=20000)
    check_preprocess(R, scene, cam, "C2-20k")


@pytest.mark.parametrize("k", [3, 4, 5, 7, 8])
def test_preprocess_parity_other_k(R, k):
    rng = np.random.default_rng(100 + k)
    centres = scenes.uniform_centres(rng, 2000)
    scene = scenes.convexes_around(rng, centres, k, 2)
    cam = scenes.orbit_camera(rng, 320, 200)
    check_preprocess(R, scene, cam, f"K={k}")


# ------------------------------------------------------------- tile lists ---

def test_tile_lists_hold_oracle_candidates_in_depth_order(R):
    import oracle
    scene, cam, _ = scenes.config2(n=4000, width=200, height=150)
    ds, rgb, st = render_gpu(R, scene, cam, want_state=True)
    ranges, ids = st.tile_lists()
    pre = oracle.preprocess(scene, cam)
    keys = np.array([c.key for c in pre], np.uint64)
    tx_n = (cam.width + 15) // 16
    rng = np.random.default_rng(0)
    tiles = rng.choice(ranges.shape[0], 25, replace=False)
    for t in tiles:
        s, e = ranges[t]
        lst = ids[s:e]
        assert len(set(lst.tolist())) == len(lst)
        order = np.lexsort((lst, keys[lst]))
        assert np.all(order == np.arange(len(lst))), "list not in (depth key, index) order"
        cand = oracle.tile_candidates(scene, cam, 16, int(t % tx_n), int(t // tx_n))
        assert set(cand.tolist()) <= set(lst.tolist()), (t, sorted(set(cand) - set(lst)))
    say(f"[lists] {len(tiles)} tiles checked, {len(ids)} pairs")
    st.release()


def test_accumulators_cleared_for_every_backward(R):
    """The backward's per-convex accumulators are cleared by the forward
    compositing kernel once the frame holds them: a second backward of the
    same forward, and the backward of later forwards on reused frames, give
    the first backward's gradients (up to the order of the float atomics)."""
    from paper_2411_14974_amd.binding import make_params
    scene, cam, _ = scenes.config2(n=3000, width=160, height=120)
    ds = dev(scene)
    dl = torch.from_numpy(np.random.default_rng(3).normal(size=(cam.height, cam.width, 3)).astype(np.float32)).cuda()

    def rel(a, b):
        return max(float((a[k].double() - b[k].double()).norm() / b[k].double().norm()) for k in NAMES)

    out, st = R.forward(ds, cam, make_params(), want_state=True)
    g1 = {k: v.clone() for k, v in R.backward(st, dl).items()}
    g2 = R.backward(st, dl)
    torch.cuda.synchronize()
    worst = rel(g2, g1)
    st.release()
    for _ in range(3):
        out, st = R.forward(ds, cam, make_params(), want_state=True)
        worst = max(worst, rel(R.backward(st, dl), g1))
        torch.cuda.synchronize()
        st.release()
    say(f"[acc] repeated backwards within {worst:.1e} of the first")
    assert worst <= 1e-5


def test_first_forward_of_a_new_context_after_another_context():
    """The pair count reaches the host through a tagged word of pinned memory;
    a new context's word may come back holding the last context's count.  A
    context that made one forward of a larger scene, closed, then a new
    context's first forward of a smaller scene: the image matches the oracle
    and the pair count is the small scene's."""
    import oracle
    from paper_2411_14974_amd.binding import Renderer
    big, cam_b, _ = scenes.config2(n=20000, width=200, height=130)
    small, cam_s, _ = scenes.config2(n=4000, width=128, height=96)
    counts = []
    for sc, cam in ((big, cam_b), (small, cam_s)):
        r = Renderer(0)
        ds, rgb, st = render_gpu(r, sc, cam, want_state=True)
        counts.append(st.stats()["pairs"])
        img = rgb.cpu().numpy()
        st.release()
        r.close()
    ref, _, _ = oracle.render(small, cam_s)
    err = float(np.abs(img.astype(np.float64) - ref).max())
    say(f"[new context] pairs {counts}, image max |gpu - oracle| {err:.2e}")
    assert counts[1] < counts[0]
    assert err <= PIX_TOL


def big_convex_scene(n=160, width=1280, height=960, seed=5):
    """Convexes stretched to 3-10x their size along a random direction (and
    2-4x across it), so that many tile rectangles exceed 64 tiles and their
    polygons fill a small part of them."""
    rng = np.random.default_rng(seed)
    sc = scenes.convexes_around(rng, scenes.uniform_centres(rng, n, (-0.6,) * 3, (0.6,) * 3), 6, 1)
    c = sc.points.astype(np.float64).mean(axis=1, keepdims=True)
    d = rng.normal(size=(n, 1, 3))
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    off = sc.points - c
    along = (off * d).sum(axis=2, keepdims=True)
    stretch = rng.uniform(3.0, 10.0, (n, 1, 1)) * along * d + rng.uniform(2.0, 4.0, (n, 1, 1)) * (off - along * d)
    pts = np.ascontiguousarray(c + stretch, dtype=np.float32)
    scene = Scene(pts, sc.delta, sc.sigma, sc.opacity, sc.sh)
    return scene, scenes.orbit_camera(rng, width, height, radius=3.0)


def test_large_rectangles_are_culled_and_keep_every_candidate(R):
    """Rectangles of more than 64 tiles drop the bands of blocks that no pixel
    centre can reach (alpha < eps_alpha there): every tile's list still holds
    the oracle's candidates, in depth order, and the image matches the
    oracle."""
    import oracle
    scene, cam = big_convex_scene()
    ds, rgb, st = render_gpu(R, scene, cam, want_state=True)
    ranges, ids = st.tile_lists()
    pre = oracle.preprocess(scene, cam)
    keys = np.array([c.key for c in pre], np.uint64)
    tx_n = (cam.width + 15) // 16
    area = np.zeros(scene.n, np.int64)
    for i, c in enumerate(pre):
        if (c.status & 0xFF) != 0:
            continue
        x0, y0, x1, y1 = c.rect
        u0, u1 = max(int(np.ceil(x0 - 0.5)), 0), min(int(np.floor(x1 - 0.5)), cam.width - 1)
        v0, v1 = max(int(np.ceil(y0 - 0.5)), 0), min(int(np.floor(y1 - 0.5)), cam.height - 1)
        if u0 <= u1 and v0 <= v1:
            area[i] = (u1 // 16 - u0 // 16 + 1) * (v1 // 16 - v0 // 16 + 1)
    big = area > 64
    per = np.bincount(ids, minlength=scene.n)
    say(f"[big rects] {int(big.sum())} rectangles over 64 tiles: {int(per[big].sum())} pairs kept of "
        f"{int(area[big].sum())} rectangle tiles")
    assert big.sum() >= 10
    assert per[big].sum() < 0.9 * area[big].sum(), "large rectangles were not culled"
    for t in range(ranges.shape[0]):
        s0, e0 = ranges[t]
        lst = ids[s0:e0]
        assert len(set(lst.tolist())) == len(lst)
        assert np.all(np.lexsort((lst, keys[lst])) == np.arange(len(lst))), t
        cand = oracle.tile_candidates(scene, cam, 16, int(t % tx_n), int(t // tx_n))
        assert set(cand.tolist()) <= set(lst.tolist()), (t, sorted(set(cand) - set(lst)))
    ref, _, _ = oracle.render(scene, cam)
    err = float(np.abs(rgb.cpu().numpy().astype(np.float64) - ref).max())
    say(f"[big rects] {ranges.shape[0]} tiles hold their candidates; image max |gpu - oracle| {err:.2e}")
    assert err <= PIX_TOL
    st.release()


# --------------------------------------------------------------- forward ----

def forward_parity(R, scene, cam, label, bg=(0.0, 0.0, 0.0)):
    import oracle
    _, rgb, _ = render_gpu(R, scene, cam, background=bg)
    ref, _, _ = oracle.render(scene, cam, mode=oracle.MODE_MATCHED, bg=bg)
    refx, _, _ = oracle.render(scene, cam, mode=oracle.MODE_EXACT, bg=bg)
    a = rgb.cpu().numpy().astype(np.float64)
    err, errx = np.abs(a - ref).max(), np.abs(a - refx).max()
    say(f"[{label}] max |gpu - oracle| matched {err:.2e}, exact {errx:.2e}")
    assert err <= PIX_TOL
    return a


def test_forward_config1(R):
    scene, cam = scenes.config1()
    forward_parity(R, scene, cam, "C1")


def test_forward_ragged_background(R):
    # 211 x 157: neither side a multiple of the 16-pixel tile
    scene, cam, _ = scenes.config2(n=15000, width=211, height=157)
    forward_parity(R, scene, cam, "C2-ragged", bg=(0.2, 0.5, 0.9))


def test_forward_mixture_small(R):
    scene, cam, _ = scenes.config3(n=40000, width=240, height=135)
    forward_parity(R, scene, cam, "C3-small")


@pytest.mark.parametrize("k,deg", [(3, 0), (4, 1), (5, 2), (8, 3)])
def test_forward_k_and_degree(R, k, deg):
    rng = np.random.default_rng(200 + k)
    centres = scenes.uniform_centres(rng, 3000)
    scene = scenes.convexes_around(rng, centres, k, deg)
    cam = scenes.orbit_camera(rng, 160, 96)
    forward_parity(R, scene, cam, f"K={k},D={deg}")


def test_forward_edge_cases(R):
    import oracle
    from paper_2411_14974_amd.binding import make_params
    # empty scene: background only
    empty = Scene(np.zeros((0, 6, 3), np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32),
                  np.zeros(0, np.float32), np.zeros((0, 16, 3), np.float32))
    cam = scenes.origin_camera(40, 24)
    _, rgb, _ = render_gpu(R, empty, cam, background=(0.1, 0.2, 0.3))
    assert np.allclose(rgb.cpu().numpy(), [0.1, 0.2, 0.3])
    # every convex behind the camera
    scene, cam = scenes.config1(n=200)
    behind = Scene(scene.points * np.array([1, 1, -1], np.float32), scene.delta, scene.sigma, scene.opacity, scene.sh)
    _, rgb, _ = render_gpu(R, behind, cam)
    assert np.abs(rgb.cpu().numpy()).max() == 0.0
    # 1 x 1 image and a convex larger than the screen
    big = Scene(np.array([[[-5, -5, 2], [5, -5, 2], [0, 5, 2.5]]], np.float32), np.array([1.0], np.float32),
                np.array([1.0], np.float32), np.array([0.7], np.float32), np.full((1, 1, 3), 0.5, np.float32))
    for w, h in ((1, 1), (33, 17)):
        c = scenes.origin_camera(w, h, focal=50.0)
        _, rgb, _ = render_gpu(R, big, c)
        ref, _, _ = oracle.render(big, c, mode=oracle.MODE_MATCHED)
        assert np.abs(rgb.cpu().numpy() - ref).max() <= PIX_TOL
    # opaque convexes drive T below t_min quickly (early termination path)
    scene, cam = scenes.config1(n=800)
    opaque = Scene(scene.points, scene.delta * 5, scene.sigma * 5, np.ones_like(scene.opacity), scene.sh)
    forward_parity(R, opaque, cam, "opaque")


# -------------------------------------------------------------- backward ----

def backward_parity(R, scene, cam, label, dl=None, bg=(0.0, 0.0, 0.0), seed=0):
    import oracle
    ds, rgb, st = render_gpu(R, scene, cam, want_state=True, background=bg)
    if dl is None:
        rng = np.random.default_rng(seed)
        dl = rng.normal(size=(cam.height, cam.width, 3)).astype(np.float32)
    g = R.backward(st, torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    ref = oracle.backward(scene, cam, dl.reshape(-1, 3), mode=oracle.MODE_MATCHED, bg=bg)
    grad_check(g, ref, label)
    st.release()


def test_backward_config1(R):
    scene, cam = scenes.config1()
    backward_parity(R, scene, cam, "C1")


def test_backward_l1_target_small_c2(R):
    # the training-step loss: mean |C - target|, its gradient computed on the GPU
    scene, cam, target = scenes.config2(n=10000, width=180, height=117)
    ds, rgb, st = render_gpu(R, scene, cam, want_state=True)
    dl = R.l1_loss_grad(rgb, torch.from_numpy(target).cuda())
    torch.cuda.synchronize()
    dl_np = dl.cpu().numpy()
    d = rgb.cpu().numpy() - target
    np.testing.assert_array_equal(dl_np, np.sign(d).astype(np.float32) / np.float32(d.size))
    backward_parity(R, scene, cam, "C2-L1", dl=dl_np)
    st.release()


def test_backward_mixture_background(R):
    scene, cam, _ = scenes.config3(n=20000, width=160, height=90)
    backward_parity(R, scene, cam, "C3-small", bg=(0.3, 0.6, 0.1), seed=3)


@pytest.mark.parametrize("k,deg", [(3, 0), (5, 1), (8, 3)])
def test_backward_k_and_degree(R, k, deg):
    rng = np.random.default_rng(300 + k)
    centres = scenes.uniform_centres(rng, 2000)
    scene = scenes.convexes_around(rng, centres, k, deg)
    cam = scenes.orbit_camera(rng, 128, 80)
    backward_parity(R, scene, cam, f"K={k},D={deg}", seed=k)


def test_backward_clamped_colours(R):
    """Colours clamped at 0 (Sec. 3.2: the SH colour is kept non-negative) in
    many convexes and channels: the backward pass takes the clamp decision of
    the forward pass, so a clamped channel passes no gradient to its SH
    coefficients, and every other gradient still matches the oracle."""
    import oracle
    rng = np.random.default_rng(4242)
    scene = scenes.convexes_around(rng, scenes.uniform_centres(rng, 3000), 6, 3)
    red, green = rng.random(scene.n) < 0.5, rng.random(scene.n) < 0.25
    scene.sh[red, 0, 0] = -3.0                  # raw red ~ 0.5 - 0.85: clamped
    scene.sh[green, 0, 1] = -1.8                # raw green near 0: clamped or not
    cam = scenes.orbit_camera(rng, 160, 100)
    cm = np.array([c.clampmask for c in oracle.preprocess(scene, cam)])
    say(f"[clamp] red clamped in {int(((cm & 1) != 0).sum())}, green in {int(((cm & 2) != 0).sum())} of {scene.n}")
    assert ((cm & 1) != 0).sum() > scene.n // 4 and ((cm & 2) != 0).sum() > 0
    ds, rgb, st = render_gpu(R, scene, cam, want_state=True)
    dl = rng.normal(size=(cam.height, cam.width, 3)).astype(np.float32)
    g = R.backward(st, torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    gsh = g["sh"].cpu().numpy()
    for bit, ch in ((1, 0), (2, 1)):
        assert np.all(gsh[(cm & bit) != 0][:, :, ch] == 0.0)
    ref = oracle.backward(scene, cam, dl.reshape(-1, 3), mode=oracle.MODE_MATCHED)
    grad_check(g, ref, "clamped colours")
    st.release()


# ------------------------------------------------ full size, sampled -------

def sampled_parity(R, scene, cam, label, npix=400, seed=0):
    """Forward on sampled pixels and backward through a dL/dC that is zero
    outside them, at the full workload size and the benchmark's launch shape."""
    import oracle
    rng = np.random.default_rng(seed)
    W, H = cam.width, cam.height
    sel = rng.choice(W * H, npix, replace=False)
    pix = np.stack([sel % W, sel // W], 1)
    say(f"[{label}] render N={scene.n} {W}x{H}")
    ds, rgb, st = render_gpu(R, scene, cam, want_state=True)
    stats = st.stats()
    a = rgb.cpu().numpy().reshape(-1, 3)[sel].astype(np.float64)
    say(f"[{label}] oracle on {npix} pixels; pairs {stats['pairs']}")
    ref, _, _ = oracle.render(scene, cam, mode=oracle.MODE_MATCHED, pixels=pix)
    err = np.abs(a - ref).max()
    say(f"[{label}] sampled max |gpu - oracle| {err:.2e}")
    assert err <= PIX_TOL
    dl = np.zeros((H * W, 3), np.float32)
    dl[sel] = rng.normal(size=(npix, 3)).astype(np.float32)
    g = R.backward(st, torch.from_numpy(dl.reshape(H, W, 3)).cuda())
    torch.cuda.synchronize()
    gref = oracle.backward(scene, cam, dl[sel], mode=oracle.MODE_MATCHED, pixels=pix)
    grad_check(g, gref, label)
    st.release()


def test_full_size_config2_sampled(R):
    scene, cam, _ = scenes.config2()
    sampled_parity(R, scene, cam, "C2-full")


# ------------------------------------------------------------- autograd ----

def test_autograd_matches_oracle_and_direct_call(R):
    """Form (3): the autograd function's image and the gradients it leaves in
    .grad match the FP64 oracle at the parity bars, and equal the direct
    calls through the C ABI."""
    import oracle
    from paper_2411_14974_amd.autograd import render
    scene, cam, _ = scenes.config2(n=3000, width=96, height=64)
    t = {k: torch.from_numpy(getattr(scene, k)).cuda().requires_grad_(True) for k in NAMES}
    rgb = render(t["points"], t["delta"], t["sigma"], t["opacity"], t["sh"], R, cam)
    w = torch.randn(rgb.shape, generator=torch.Generator().manual_seed(7)).cuda()
    (rgb * w).sum().backward()
    torch.cuda.synchronize()
    ref, _, _ = oracle.render(scene, cam, mode=oracle.MODE_MATCHED)
    err = np.abs(rgb.detach().cpu().numpy() - ref).max()
    say(f"[autograd] max |rgb - oracle| {err:.2e}")
    assert err <= PIX_TOL
    gref = oracle.backward(scene, cam, w.cpu().numpy().reshape(-1, 3), mode=oracle.MODE_MATCHED)
    grad_check({k: t[k].grad for k in NAMES}, gref, "autograd .grad vs oracle")
    ds, rgb2, st = render_gpu(R, scene, cam, want_state=True)
    g = R.backward(st, w)
    torch.cuda.synchronize()
    assert torch.equal(rgb.detach(), rgb2)
    for k in NAMES:
        torch.testing.assert_close(t[k].grad, g[k], rtol=1e-5, atol=1e-7)
    st.release()


def test_work_counters_against_the_oracle(R):
    """cs_state_counters: the pairs past the max-line test bound the pairs the
    oracle composites (every pixel's contributors, matched mode) and are
    bounded by the pairs tested; the backward walk (up to each pixel's last
    contributor) sees a subset of the forward's (which walks on until T falls
    below t_min); the mean hull size lies in [3, K]; lane utilisation in (0, 1]."""
    import oracle
    from paper_2411_14974_amd.binding import DeviceScene, make_params
    scene, cam, _ = scenes.config3(n=40000, width=240, height=135)
    ds = DeviceScene.from_scene(scene, "cuda:0")
    rgb, st = R.forward(ds, cam, make_params(), want_state=True)
    dl = torch.ones_like(rgb)
    R.backward(st, dl)
    torch.cuda.synchronize()
    c = st.counters()
    _, _, nref = oracle.render(scene, cam, mode=oracle.MODE_MATCHED)
    contrib = int(nref.sum())
    T_mean = c["sum_T_full"] / c["full_bwd"]
    util = c["full_bwd"] / (64 * c["wave_evals"])
    print(f"[counters] {c}; oracle contributors {contrib}; mean T {T_mean:.3f}; lane utilisation {util:.3f}", flush=True)
    assert contrib <= c["full_bwd"] <= c["full"] <= c["tested"] <= 256 * c["pairs"]
    assert 3.0 <= T_mean <= scene.k
    assert 0.0 < util <= 1.0
    st.release()
