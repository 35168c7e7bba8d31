"""Density control on the GPU (split / prune, paper Sec. 3.3) against the oracle.

Bars: the decisions, the output order and the source indices bit-exact (both
sides decide in float32 in the same order); copied values (delta, SH, kept
convexes) bit-exact; the children's sigma and opacity bit-exact (one float32
rounding of an exact product on both sides); the children's points within
2e-6 of the oracle's float64 geometry (a few float32 roundings of O(1)
coordinates).  The statistic accumulated after a backward pass equals |dL/dsigma|
on the convexes that reached a tile of the view.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2411_14974_amd import scenes  # noqa: E402

PTS_TOL = 2e-6


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    from paper_2411_14974_amd.binding import Renderer
    r = Renderer(0)
    yield r
    r.close()


def params(**kw):
    from paper_2411_14974_amd.binding import make_densify_params
    return make_densify_params(**kw)


def statistic(rng, n, frac_split):
    denom = rng.integers(0, 4, n).astype(np.float32)
    mean = np.where(rng.random(n) < frac_split, rng.uniform(5e-6, 1e-4, n), rng.uniform(0, 3e-6, n))
    return (mean * denom).astype(np.float32), denom


def run_and_compare(R, scene, accum, denom, label, **kw):
    from oracle import densify as D
    from paper_2411_14974_amd.binding import DeviceScene
    p = params(**kw)
    ds = DeviceScene.from_scene(scene, "cuda:0")
    a, d = torch.from_numpy(accum).cuda(), torch.from_numpy(denom).cuda()
    out, src = R.densify(ds, a, d, p)
    torch.cuda.synchronize()
    ref = D.densify(scene, accum, denom, p.opacity_min, p.size_max, p.split_threshold, p.child_scale,
                    p.child_sigma_scale, p.child_opacity_scale)
    pts, dl, sg, op, sh, rsrc = ref
    say(f"[{label}] {scene.n} -> {out.n} convexes")
    assert out.n == pts.shape[0]
    assert np.array_equal(src.cpu().numpy(), rsrc)
    np.testing.assert_array_equal(out.delta.cpu().numpy(), dl.astype(np.float32))
    np.testing.assert_array_equal(out.sigma.cpu().numpy(), sg.astype(np.float32))
    np.testing.assert_array_equal(out.opacity.cpu().numpy(), op.astype(np.float32))
    np.testing.assert_array_equal(out.sh.cpu().numpy(), sh)
    err = float(np.abs(out.points.cpu().numpy().astype(np.float64) - pts).max()) if out.n else 0.0
    say(f"[{label}] max |points - oracle| {err:.1e}")
    assert err <= PTS_TOL
    return out


def test_densify_mixture_matches_oracle(R):
    rng = np.random.default_rng(61)
    scene = scenes.convexes_around(rng, scenes.gmm_centres(rng, 50_000), 6, 3)
    scene.opacity[rng.random(scene.n) < 0.05] = 0.01               # some nearly transparent
    accum, denom = statistic(rng, scene.n, 0.08)
    # size limit inside the radius distribution: some convexes too large
    run_and_compare(R, scene, accum, denom, "mixture 50k", size_max=0.12)


@pytest.mark.parametrize("k,deg,n", [(3, 0, 1001), (5, 1, 4097), (8, 2, 777)])
def test_densify_other_k_degree_ragged(R, k, deg, n):
    rng = np.random.default_rng(70 + k)
    scene = scenes.convexes_around(rng, scenes.uniform_centres(rng, n), k, deg)
    accum, denom = statistic(rng, n, 0.3)
    run_and_compare(R, scene, accum, denom, f"K={k} D={deg} n={n}", size_max=0.15, child_scale=0.6,
                    child_sigma_scale=2.0, child_opacity_scale=0.3)


def test_densify_edge_cases(R):
    from paper_2411_14974_amd.binding import CS_EOVERFLOW, CSError, DeviceScene
    rng = np.random.default_rng(80)
    scene = scenes.convexes_around(rng, scenes.uniform_centres(rng, 300), 6, 1)
    ones = np.ones(300, np.float32)
    # nothing passes: identity
    out = run_and_compare(R, scene, np.zeros(300, np.float32), ones, "identity", opacity_min=0.0, size_max=1e9,
                          split_threshold=1e9)
    assert out.n == 300
    # everything pruned: empty result
    out = run_and_compare(R, scene, ones, ones, "all pruned", opacity_min=2.0)
    assert out.n == 0
    # everything split
    out = run_and_compare(R, scene, ones, ones, "all split", opacity_min=0.0, size_max=1e9, split_threshold=0.5)
    assert out.n == 300 * 6
    # too small a capacity: overflow reported with the needed count (the binding grows and retries)
    ds = DeviceScene.from_scene(scene, "cuda:0")
    a, d = torch.from_numpy(ones).cuda(), torch.from_numpy(ones).cuda()
    with pytest.raises(CSError) as ei:
        from paper_2411_14974_amd import binding
        so = binding.SceneOut(0, 0, 0, 0, 0, 0)
        n_out = binding.C.c_int64()
        p = params(opacity_min=0.0, size_max=1e9, split_threshold=0.5)
        rc = binding.lib().cs_densify(R.ctx, binding.C.byref(ds.struct()), a.data_ptr(), d.data_ptr(),
                                      binding.C.byref(p), 10, binding.C.byref(so), binding.C.byref(n_out), None)
        assert n_out.value == 1800
        binding._check(rc)
    assert ei.value.code == CS_EOVERFLOW
    out, src = R.densify(ds, a, d, params(opacity_min=0.0, size_max=1e9, split_threshold=0.5), capacity=10)
    assert out.n == 1800
    # empty scene
    empty = scenes.Scene(np.zeros((0, 6, 3), np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32),
                         np.zeros(0, np.float32), np.zeros((0, 4, 3), np.float32))
    out, src = R.densify(DeviceScene.from_scene(empty, "cuda:0"), torch.zeros(0, device="cuda"),
                         torch.zeros(0, device="cuda"))
    assert out.n == 0


def test_accumulate_after_backward(R):
    from paper_2411_14974_amd.binding import DeviceScene, make_params
    scene, cam, target = scenes.config2(n=20000, width=200, height=130)
    ds = DeviceScene.from_scene(scene, "cuda:0")
    img, st = R.forward(ds, cam, make_params(), want_state=True)
    dl = R.l1_loss_grad(img, torch.from_numpy(target).cuda())
    g = R.backward(st, dl)
    accum = torch.full((scene.n,), 0.25, device="cuda")
    denom = torch.full((scene.n,), 1.0, device="cuda")
    R.densify_accumulate(st, g["sigma"], accum, denom)
    torch.cuda.synchronize()
    ranges, ids = st.tile_lists()
    seen = np.zeros(scene.n, bool)
    seen[np.unique(ids)] = True
    a, d = accum.cpu().numpy(), denom.cpu().numpy()
    gs = np.abs(g["sigma"].cpu().numpy())
    assert np.array_equal(d, np.where(seen, 2.0, 1.0).astype(np.float32))
    np.testing.assert_array_equal(a, np.where(seen, np.float32(0.25) + gs, np.float32(0.25)).astype(np.float32))
    say(f"[accumulate] {int(seen.sum())} of {scene.n} convexes reached a tile")
    st.release()
