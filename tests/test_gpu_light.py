"""16-bit scene parameters (the paper's light model, Sec. 4.2), through the C ABI.

The kernels convert every stored 16-bit value to float32 exactly and then run
the float32 arithmetic, so a float16 or bfloat16 scene must render bit for bit
like the float32 scene holding the same (rounded) values, and its gradients
(float32 atomics: equal up to summation order) must match that scene's.  The
oracle, fed those rounded values, bounds both at the usual parity tolerances.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2411_14974_amd import scenes  # noqa: E402

PIX_TOL = 1e-4
GRAD_TOL = 1e-3
NAMES = ("points", "delta", "sigma", "opacity", "sh")
FORMATS = (("f16", torch.float16), ("bf16", torch.bfloat16))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    from paper_2411_14974_amd.binding import Renderer
    r = Renderer(0)
    yield r
    r.close()


def dev(scene, dtype=torch.float32):
    from paper_2411_14974_amd.binding import DeviceScene
    return DeviceScene.from_scene(scene, "cuda:0", dtype=dtype)


def rel_gap(a, b):
    a = a.detach().double().cpu().numpy().ravel()
    b = np.asarray(b.detach().double().cpu().numpy() if hasattr(b, "detach") else b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def grad_check(g, ref, label):
    for k in NAMES:
        a = g[k].detach().cpu().numpy().astype(np.float64).ravel()
        b = np.asarray(ref[k], np.float64).ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        rms = np.sqrt(np.mean(b * b))
        el = float((np.abs(a - b) / np.maximum(np.abs(b), 1e-2 * rms + 1e-300)).max())
        say(f"[{label}] {k}: rel-L2 {rel:.1e}, worst element {el:.1e}")
        assert rel <= GRAD_TOL and el <= GRAD_TOL, (label, k, rel, el)


@pytest.mark.parametrize("fmt,dtype", FORMATS)
def test_16bit_scene_renders_as_its_float32_values(R, fmt, dtype):
    from paper_2411_14974_amd.binding import make_params
    # ragged size, several tiles, SH degree 3
    scene, cam, _ = scenes.config2(n=20000, width=227, height=141)
    d16 = dev(scene, dtype)
    d32 = dev(scene.stored(fmt))
    assert d16.points.dtype == dtype and d16.points.element_size() == 2
    img16, st16 = R.forward(d16, cam, make_params(), want_state=True)
    img32, st32 = R.forward(d32, cam, make_params(), want_state=True)
    torch.cuda.synchronize()
    assert torch.equal(img16, img32)
    assert st16.stats() == st32.stats()
    rng = np.random.default_rng(11)
    dl = torch.from_numpy(rng.normal(size=(cam.height, cam.width, 3)).astype(np.float32)).cuda()
    g16 = R.backward(st16, dl)
    g32 = R.backward(st32, dl)
    torch.cuda.synchronize()
    for k in NAMES:
        assert g16[k].dtype == torch.float32
        gap = rel_gap(g16[k], g32[k])
        assert gap <= 1e-5, (fmt, k, gap)
    say(f"[{fmt}] image bit-identical to the float32 scene of its values; pairs {st16.stats()['pairs']}")
    st16.release()
    st32.release()


@pytest.mark.parametrize("fmt,dtype", FORMATS)
def test_16bit_scene_matches_oracle(R, fmt, dtype):
    import oracle
    from paper_2411_14974_amd.binding import make_params
    scene, cam, _ = scenes.config3(n=20000, width=160, height=90)
    # Rounding to 16 bits puts some convexes' points on top of each other or
    # on a line (bfloat16: ~0.7 % of these convexes, float16: ~0.01 %).  Their
    # hull is ill-posed: the oracle flags them degenerate and, as for any
    # degenerate convex, they are left out of the comparison.
    status = np.array([c.status for c in oracle.preprocess(scene.stored(fmt), cam)])
    keep = np.nonzero((status & oracle.DEGENERATE) == 0)[0]
    say(f"[{fmt}] {scene.n - keep.size} degenerate convexes left out")
    scene = scene.subset(keep)
    held = scene.stored(fmt)
    d16 = dev(scene, dtype)
    img, st = R.forward(d16, cam, make_params(background=(0.2, 0.1, 0.4)), want_state=True)
    torch.cuda.synchronize()
    ref, _, _ = oracle.render(held, cam, mode=oracle.MODE_MATCHED, bg=(0.2, 0.1, 0.4))
    err = float(np.abs(img.cpu().numpy().astype(np.float64) - ref).max())
    say(f"[{fmt}] max |gpu - oracle| {err:.2e}")
    assert err <= PIX_TOL
    rng = np.random.default_rng(12)
    dl = rng.normal(size=(cam.height, cam.width, 3)).astype(np.float32)
    g = R.backward(st, torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    gref = oracle.backward(held, cam, dl.reshape(-1, 3), mode=oracle.MODE_MATCHED, bg=(0.2, 0.1, 0.4))
    grad_check(g, gref, fmt)
    st.release()


@pytest.mark.parametrize("k,deg", [(3, 0), (5, 2), (8, 1)])
def test_16bit_scene_other_k_and_degree(R, k, deg):
    """The non-vectorised SH loads (degrees 0-2) and odd point counts."""
    from paper_2411_14974_amd.binding import make_params
    rng = np.random.default_rng(500 + k)
    scene = scenes.convexes_around(rng, scenes.uniform_centres(rng, 3000), k, deg)
    cam = scenes.orbit_camera(rng, 150, 90)
    for fmt, dtype in FORMATS:
        img16, st16 = R.forward(dev(scene, dtype), cam, make_params(), want_state=True)
        img32, st32 = R.forward(dev(scene.stored(fmt)), cam, make_params(), want_state=True)
        torch.cuda.synchronize()
        assert torch.equal(img16, img32), (fmt, k, deg)
        dl = torch.from_numpy(rng.normal(size=(cam.height, cam.width, 3)).astype(np.float32)).cuda()
        g16, g32 = R.backward(st16, dl), R.backward(st32, dl)
        torch.cuda.synchronize()
        for name in NAMES:
            assert rel_gap(g16[name], g32[name]) <= 1e-5, (fmt, k, deg, name)
        st16.release()
        st32.release()


def test_16bit_batched_graph_equals_per_view(R):
    from paper_2411_14974_amd.binding import FLAG_GRAPH, make_params
    rng = np.random.default_rng(4100)
    scene = scenes.convexes_around(rng, scenes.gmm_centres(rng, 15000), 6, 3)
    cams = [scenes.orbit_camera(rng, *wh) for wh in ((200, 120), (97, 61), (256, 144))]
    d16 = dev(scene, torch.float16)
    ref = []
    for c in cams:
        img, _ = R.forward(d16, c, make_params())
        ref.append(img)
    for rep in range(3):  # eager sizing frame, then graph replays
        outs, st = R.forward_batch(d16, cams, make_params(flags=FLAG_GRAPH), want_state=True)
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), rep
        assert R.batch_check(st) == 0
        st.release()
    say("[f16 batch] graph replays equal per-view renders")


def test_autograd_with_half_parameters(R):
    from paper_2411_14974_amd.autograd import render
    scene, cam, _ = scenes.config2(n=3000, width=96, height=64)
    t = {k: torch.from_numpy(getattr(scene, k)).cuda().half().requires_grad_(True) for k in NAMES}
    rgb = render(t["points"], t["delta"], t["sigma"], t["opacity"], t["sh"], R, cam)
    w = torch.randn_like(rgb)
    (rgb * w).sum().backward()
    t32 = {k: t[k].detach().float().requires_grad_(True) for k in NAMES}
    rgb32 = render(t32["points"], t32["delta"], t32["sigma"], t32["opacity"], t32["sh"], R, cam)
    (rgb32 * w).sum().backward()
    assert torch.equal(rgb.detach(), rgb32.detach())
    for k in NAMES:
        assert t[k].grad.dtype == torch.float16
        torch.testing.assert_close(t[k].grad, t32[k].grad.half(), rtol=2e-3, atol=1e-6)
