"""Batched multi-view rendering, hipGraph replay, tile configurations and the
autotuner (through the C ABI).

A batch renders every view with the same per-pixel evaluation as the plain
one-view path, so its images are bit-identical to per-view renders; its
gradients are the sum of the per-view gradients (float atomics: equal up to
summation order).  The tile size and the tile schedule change which
(pixel, convex) pairs are tested, never which ones contribute, so images are
bit-identical across them too.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2411_14974_amd import scenes  # noqa: E402

NAMES = ("points", "delta", "sigma", "opacity", "sh")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def R():
    from paper_2411_14974_amd.binding import Renderer
    r = Renderer(0)
    yield r
    r.close()


def dev(scene):
    from paper_2411_14974_amd.binding import DeviceScene
    return DeviceScene.from_scene(scene, "cuda:0")


def grad_gap(a, b):
    """(relative L2 gap, worst element gap relative to max(|b|, 1e-2 rms(b)))."""
    a = a.detach().double().cpu().numpy().ravel()
    b = b.detach().double().cpu().numpy().ravel()
    rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
    return (float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)),
            float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-2 * rms + 1e-300))) if b.size else 0.0)


def grads_close(a, b, tol=1e-3):
    """Two float-atomic sums of the same terms in different orders: within the
    parity tolerance per element (floor 1e-2 rms) and 1e-5 in norm."""
    rel, worst = grad_gap(a, b)
    return rel <= 1e-5 and worst <= tol


def small_batch(n=20000, views=5, seed=0, res=((200, 120), (97, 61), (256, 144))):
    rng = np.random.default_rng(4000 + seed)
    centres = scenes.gmm_centres(rng, n)
    scene = scenes.convexes_around(rng, centres, 6, 3)
    cams = [scenes.orbit_camera(rng, *res[i % len(res)]) for i in range(views)]
    return scene, cams


def plain_views(R, ds, cams, **kw):
    from paper_2411_14974_amd.binding import make_params
    outs = []
    for c in cams:
        img, _ = R.forward(ds, c, make_params(**kw))
        outs.append(img)
    torch.cuda.synchronize()
    return outs


def test_batch_forward_equals_per_view(R):
    from paper_2411_14974_amd.binding import make_params
    scene, cams = small_batch()
    ds = dev(scene)
    ref = plain_views(R, ds, cams)
    outs, st = R.forward_batch(ds, cams, make_params(), want_state=True)
    torch.cuda.synchronize()
    for v, (a, b) in enumerate(zip(outs, ref)):
        assert torch.equal(a, b), v
    say(f"[batch] {len(cams)} views bit-identical to per-view renders, pairs {st.stats()['pairs']}")
    st.release()


def test_batch_backward_sums_views_and_matches_oracle(R):
    import oracle
    from paper_2411_14974_amd.binding import make_params
    scene, cams = small_batch(n=6000, views=3, seed=1, res=((96, 64), (80, 57), (120, 72)))
    ds = dev(scene)
    rng = np.random.default_rng(5)
    dls = [torch.from_numpy(rng.normal(size=(c.height, c.width, 3)).astype(np.float32)).cuda() for c in cams]
    outs, st = R.forward_batch(ds, cams, make_params(), want_state=True)
    g = R.backward_batch(st, dls)
    torch.cuda.synchronize()
    total = {k: torch.zeros_like(g[k]) for k in NAMES}
    ref = {k: 0.0 for k in NAMES}
    for c, d in zip(cams, dls):
        _, s1 = R.forward(ds, c, make_params(), want_state=True)
        g1 = R.backward(s1, d)
        torch.cuda.synchronize()
        for k in NAMES:
            total[k] += g1[k]
        o = oracle.backward(scene, c, d.cpu().numpy().reshape(-1, 3))
        for k in NAMES:
            ref[k] = ref[k] + o[k]
        s1.release()
    for k in NAMES:
        a, b = g[k].cpu().numpy().astype(np.float64), total[k].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b), k
        rel = np.linalg.norm(a.ravel() - ref[k].ravel()) / np.linalg.norm(ref[k])
        say(f"[batch-bwd] {k}: vs sum of views {np.linalg.norm(a - b) / np.linalg.norm(b):.1e}, vs oracle {rel:.1e}")
        assert rel <= 1e-3, k
    st.release()


@pytest.mark.parametrize("k,deg,dtype", [(4, 1, "f32"), (8, 2, "f32"), (3, 0, "f32"), (6, 3, "f16"), (5, 2, "bf16")])
def test_batch_backward_other_k_degree_storage(R, k, deg, dtype):
    """The several-view backward keeps degree-3 SH coefficients in registers
    (float32 or 16-bit storage) and reads lower degrees row by row: every form
    sums to the per-view gradients."""
    from paper_2411_14974_amd.binding import DeviceScene, make_params
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    rng = np.random.default_rng(4300 + 10 * k + deg)
    scene = scenes.convexes_around(rng, scenes.uniform_centres(rng, 3001), k, deg)
    cams = [scenes.orbit_camera(rng, *wh) for wh in ((96, 64), (81, 57), (120, 72), (64, 48))]
    ds = DeviceScene.from_scene(scene, "cuda:0", dtype=tdt)
    dls = [torch.from_numpy(rng.normal(size=(c.height, c.width, 3)).astype(np.float32)).cuda() for c in cams]
    _, st = R.forward_batch(ds, cams, make_params(), want_state=True)
    g = R.backward_batch(st, dls)
    torch.cuda.synchronize()
    total = {name: torch.zeros_like(g[name]) for name in NAMES}
    for c, d in zip(cams, dls):
        _, s1 = R.forward(ds, c, make_params(), want_state=True)
        g1 = R.backward(s1, d)
        torch.cuda.synchronize()
        for name in NAMES:
            total[name] += g1[name]
        s1.release()
    for name in NAMES:
        a, b = g[name].cpu().numpy().astype(np.float64), total[name].cpu().numpy().astype(np.float64)
        gap = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        assert gap <= 1e-5, (k, deg, dtype, name, gap)
    say(f"[batch-bwd K={k} D={deg} {dtype}] equals the sum of per-view gradients")
    st.release()


@pytest.mark.parametrize("tile,longest", [(8, 0), (32, 0), (16, 1), (8, 1), (32, 1)])
def test_tile_configs_identical_and_match_oracle(R, tile, longest):
    import oracle
    from paper_2411_14974_amd.binding import FLAG_LONGEST_FIRST, make_params
    scene, cam, _ = scenes.config2(n=12000, width=203, height=131)
    ds = dev(scene)
    ref16 = plain_views(R, ds, [cam])[0]
    flags = FLAG_LONGEST_FIRST if longest else 0
    img, st = R.forward(ds, cam, make_params(tile=tile, flags=flags), want_state=True)
    torch.cuda.synchronize()
    assert torch.equal(img, ref16)
    o, _, _ = oracle.render(scene, cam, mode=oracle.MODE_MATCHED)
    assert np.abs(img.cpu().numpy() - o).max() <= 1e-4
    rng = np.random.default_rng(tile + longest)
    dl = rng.normal(size=(cam.height, cam.width, 3)).astype(np.float32)
    g = R.backward(st, torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    ref = oracle.backward(scene, cam, dl.reshape(-1, 3))
    for k in NAMES:
        a = g[k].cpu().numpy().astype(np.float64).ravel()
        rel = np.linalg.norm(a - ref[k].ravel()) / np.linalg.norm(ref[k])
        assert rel <= 1e-3, (tile, longest, k, rel)
    say(f"[tile {tile}, longest {longest}] identical image, grads within 1e-3: pairs {st.stats()['pairs']}")
    st.release()


def test_graph_replay_matches_eager_with_changing_cameras(R):
    from paper_2411_14974_amd.binding import FLAG_GRAPH, make_params
    scene, cams_a = small_batch(n=15000, views=4, seed=2)
    _, cams_b = small_batch(n=15000, views=4, seed=3)  # same resolutions, other poses
    ds = dev(scene)
    pg = make_params(flags=FLAG_GRAPH)
    rng = np.random.default_rng(9)
    grads = {k: torch.empty_like(getattr(ds, k)) for k in NAMES}
    for rep, cams in enumerate([cams_a, cams_a, cams_b, cams_a, cams_b, cams_b]):
        outs, st = R.forward_batch(ds, cams, pg, want_state=True)
        dls = [torch.from_numpy(rng.normal(size=(c.height, c.width, 3)).astype(np.float32)).cuda() for c in cams]
        R.backward_batch(st, dls, grads=grads)
        torch.cuda.synchronize()
        # eager reference, with the program's own work in between replays
        ref_outs, st2 = R.forward_batch(ds, cams, make_params(), want_state=True)
        g2 = R.backward_batch(st2, dls)
        torch.cuda.synchronize()
        for a, b in zip(outs, ref_outs):
            assert torch.equal(a, b), rep
        # two eager runs: the size of summation-order noise alone
        ref_outs2, st3 = R.forward_batch(ds, cams, make_params(), want_state=True)
        g3 = R.backward_batch(st3, dls)
        torch.cuda.synchronize()
        for k in NAMES:
            say(f"[graph rep {rep}] {k}: graph vs eager {grad_gap(grads[k], g2[k])}, "
                f"eager vs eager {grad_gap(g3[k], g2[k])}")
            assert grads_close(grads[k], g2[k]), (rep, k, grad_gap(grads[k], g2[k]))
        st3.release()
        assert R.batch_check(st) == 0
        st.release()
        st2.release()
    say("[graph] 6 replays (2 camera sets) equal eager forward and backward")


def test_graph_backward_twice_after_one_forward(R):
    """The batched graphs clear the backward's accumulators in the forward's
    compositing once the frame holds them; a second backward of the same
    forward (the graph with its own clearing pass) gives the first's
    gradients, and so does the backward of a later forward."""
    from paper_2411_14974_amd.binding import FLAG_GRAPH, make_params
    scene, cams = small_batch(n=15000, views=4, seed=4)
    ds = dev(scene)
    pg = make_params(flags=FLAG_GRAPH)
    rng = np.random.default_rng(5)
    dls = [torch.from_numpy(rng.normal(size=(c.height, c.width, 3)).astype(np.float32)).cuda() for c in cams]
    ref = None
    for rep in range(3):  # frame creation, capture with clearing, replay
        outs, st = R.forward_batch(ds, cams, pg, want_state=True)
        g1 = {k: v.clone() for k, v in R.backward_batch(st, dls).items()}
        g2 = R.backward_batch(st, dls)
        torch.cuda.synchronize()
        if ref is None:
            ref = g1
        for k in NAMES:
            assert grads_close(g2[k], g1[k]), (rep, k, grad_gap(g2[k], g1[k]))
            assert grads_close(g1[k], ref[k]), (rep, k, grad_gap(g1[k], ref[k]))
        assert R.batch_check(st) == 0
        st.release()
    say("[graph] repeated backwards of one forward and later forwards agree")


def test_graph_overflow_is_reported_and_recovers(R):
    from paper_2411_14974_amd.binding import CS_EOVERFLOW, FLAG_GRAPH, Camera, make_camera, make_params
    scene, cams = small_batch(n=20000, views=2, seed=4, res=((256, 160),))
    ds = dev(scene)
    far = []
    for c in cams:  # move the cameras back: few pairs in the first (sizing) frame
        cf = make_camera(c)
        cf.t[2] = cf.t[2] + 6.0
        far.append(cf)
    pg = make_params(flags=FLAG_GRAPH)
    outs, st = R.forward_batch(ds, far, pg, want_state=True)
    assert R.batch_check(st) == 0
    st.release()
    outs, st = R.forward_batch(ds, cams, pg, want_state=True)  # many more pairs: overflow
    assert R.batch_check(st) == CS_EOVERFLOW
    st.release()
    outs, st = R.forward_batch(ds, cams, pg, want_state=True)  # buffers have grown
    assert R.batch_check(st) == 0
    torch.cuda.synchronize()
    ref = plain_views(R, ds, cams)
    for a, b in zip(outs, ref):
        assert torch.equal(a, b)
    st.release()
    say("[graph] overflow reported, re-render after growth matches eager")


def test_autotune_and_autotuned_batch(R):
    from paper_2411_14974_amd.binding import FLAG_AUTOTUNE, FLAG_GRAPH, make_params
    scene, cams = small_batch(n=20000, views=4, seed=6)
    ds = dev(scene)
    t = R.autotune(ds, cams)
    say(f"[autotune] {t}")
    assert t["tile"] in (8, 16, 32) and t["longest_first"] in (0, 1) and t["digit_bits"] in (6, 8)
    assert 0 < t["ms"] <= t["ms_default"]
    outs, st = R.forward_batch(ds, cams, make_params(flags=FLAG_AUTOTUNE | FLAG_GRAPH), want_state=True)
    torch.cuda.synchronize()
    ref = plain_views(R, ds, cams)
    for a, b in zip(outs, ref):
        assert torch.equal(a, b)
    st.release()


def test_eager_frame_reuse_with_more_pairs_matches_fresh(R):
    """A reused frame runs the post-count tail on the device-side count; when
    the new view needs more pairs than its buffers hold, the tail runs again
    with grown buffers, and the image equals a fresh renderer's."""
    from paper_2411_14974_amd.binding import Renderer, make_camera, make_params
    scene, cams = small_batch(n=20000, views=1, seed=8, res=((256, 160),))
    ds = dev(scene)
    near = cams[0]
    far = make_camera(near)
    far.t[2] = far.t[2] + 6.0  # few pairs: the cached frame gets small pair buffers
    R.forward(ds, far, make_params())
    img, st = R.forward(ds, near, make_params(), want_state=True)  # reuses that frame, overflows
    torch.cuda.synchronize()
    fresh = Renderer(0)
    try:
        ref, st2 = fresh.forward(ds, near, make_params(), want_state=True)
        torch.cuda.synchronize()
        assert torch.equal(img, ref)
        assert st.stats()["pairs"] == st2.stats()["pairs"]
        say(f"[reuse] {st.stats()['pairs']} pairs after growing a reused frame: image equals a fresh render")
        st2.release()
    finally:
        fresh.close()
    st.release()
