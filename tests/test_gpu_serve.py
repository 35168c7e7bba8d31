"""Serving: continuous batching of view requests against resident scenes.

Each served image must equal the same view rendered alone by the plain path
(bit-identical: a batch evaluates every pixel exactly like a single view),
whatever batch it landed in, and match the FP64 oracle within 1e-4 (one image
of each scene and resolution); admission and queue limits return their codes.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2411_14974_amd import scenes  # noqa: E402


@pytest.fixture(scope="module")
def R():
    from paper_2411_14974_amd.binding import Renderer
    r = Renderer(0)
    yield r
    r.close()


def host_scenes():
    out = []
    for i, n in enumerate((8000, 20000)):
        rng = np.random.default_rng(5000 + i)
        out.append(scenes.convexes_around(rng, scenes.gmm_centres(rng, n), 6, 3))
    return out


def two_scenes():
    from paper_2411_14974_amd.binding import DeviceScene
    return [DeviceScene.from_scene(s, "cuda:0") for s in host_scenes()]


def test_served_equals_alone_in_the_mix(R):
    import oracle
    from paper_2411_14974_amd.binding import make_params
    host = host_scenes()
    ds = two_scenes()
    R.serve_start(workers=3, max_batch=6, start_paused=True)
    try:
        sids = [R.scene_register(d) for d in ds]
        rng = np.random.default_rng(11)
        res = ((256, 256), (160, 90), (320, 180))
        reqs = []
        for i in range(20):
            s = int(rng.integers(0, 2))
            cam = scenes.orbit_camera(rng, *res[int(rng.integers(0, 3))])
            out = torch.full((cam.height, cam.width, 3), -1.0, device="cuda:0")
            reqs.append((s, cam, out, R.serve_submit(sids[s], cam, out)))
        R.serve_resume()  # everything queued before the workers start: batches form
        lat = [R.serve_wait(rid) for _, _, _, rid in reqs]
        st = R.serve_stats()
        print(f"[serve] stats {st}, latency ms max {max(lat):.2f}", flush=True)
        assert st["completed"] == 20 and st["failed"] == 0 and st["mean_batch"] > 1.0
        torch.cuda.synchronize()
        for s, cam, out, _ in reqs:
            alone, _ = R.forward(ds[s], cam, make_params())
            torch.cuda.synchronize()
            assert torch.equal(out, alone)
        # served images against the FP64 oracle: both scenes, every resolution
        seen = {}
        for s, cam, out, _ in reqs:
            seen.setdefault((s, cam.width, cam.height), []).append((cam, out))
        assert len(seen) == 6, sorted(seen)
        for (s, w, h), lst in sorted(seen.items()):
            cam, out = lst[0]
            ref, _, _ = oracle.render(host[s], cam, mode=oracle.MODE_MATCHED)
            err = float(np.abs(out.cpu().numpy() - ref).max())
            print(f"[serve] scene {s} {w}x{h}: max |served - oracle| {err:.2e}", flush=True)
            assert err <= 1e-4
        # while requests run, more arrive and join later batches
        more = []
        for i in range(30):
            cam = scenes.orbit_camera(rng, 128, 96)
            out = torch.empty((96, 128, 3), device="cuda:0")
            more.append((cam, out, R.serve_submit(sids[1], cam, out)))
        for cam, out, rid in more:
            R.serve_wait(rid)
        torch.cuda.synchronize()
        for cam, out, _ in more[::5]:
            alone, _ = R.forward(ds[1], cam, make_params())
            torch.cuda.synchronize()
            assert torch.equal(out, alone)
    finally:
        R.serve_stop()


def test_admission_and_queue_limits(R):
    from paper_2411_14974_amd.binding import CS_EBUSY, CS_EINVAL, CS_ENOMEM, make_camera
    ds = two_scenes()
    cam = make_camera(scenes.origin_camera(64, 64))
    out = torch.empty((64, 64, 3), device="cuda:0")
    # a budget no request fits
    R.serve_start(workers=1, max_batch=4, hbm_budget_bytes=4096)
    try:
        sid = R.scene_register(ds[0])
        rc, _ = R.serve_submit_raw(sid, cam, out.data_ptr())
        assert rc == CS_ENOMEM
        rc, _ = R.serve_submit_raw(sid + 100, cam, out.data_ptr())
        assert rc == CS_EINVAL
    finally:
        R.serve_stop()
    # queue limit while paused; stop fails what is still queued
    R.serve_start(workers=1, max_batch=4, max_queue=2, start_paused=True)
    sid = R.scene_register(ds[0])
    rc1, r1 = R.serve_submit_raw(sid, cam, out.data_ptr())
    rc2, r2 = R.serve_submit_raw(sid, cam, out.data_ptr())
    rc3, _ = R.serve_submit_raw(sid, cam, out.data_ptr())
    assert (rc1, rc2, rc3) == (0, 0, CS_EBUSY)
    assert R.serve_stats()["queued"] == 2
    R.serve_stop()


def estimate_bytes(n, k, views, pixels):
    """The server's admission estimate of a batch (per instance the record
    and 60 bytes of keys and binning, a quarter more for capacity rounding,
    16 pairs of 16 bytes; 8 bytes per pixel; 2 MiB)."""
    rec = (48 + 24 * k + 15) & ~15
    inst = n * views
    return int(inst * (rec + 60) * 1.25) + inst * 16 * 16 + pixels * 8 + (2 << 20)


def test_frames_count_against_the_budget_and_are_reused(R):
    """Frames (idle or running) never hold more device memory than the budget
    when every batch fits it alone; with no budget, a second round of the same
    request mix allocates no frame."""
    from paper_2411_14974_amd.binding import DeviceScene
    sizes = (20000, 40000, 60000)
    ds = []
    for i, n in enumerate(sizes):
        rng = np.random.default_rng(5100 + i)
        ds.append(DeviceScene.from_scene(scenes.convexes_around(rng, scenes.gmm_centres(rng, n), 6, 3), "cuda:0"))
    W, H = 320, 180
    budget = int(2.5 * estimate_bytes(max(sizes), 6, 2, 2 * W * H))

    def round_of(sids, rng, count, resume=False):
        outs = [torch.empty((H, W, 3), device="cuda:0") for _ in range(count)]
        ids = [R.serve_submit(sids[int(rng.integers(0, len(sids)))], scenes.orbit_camera(rng, W, H), o)
               for o in outs]
        if resume:
            R.serve_resume()
        for rid in ids:
            R.serve_wait(rid)
        return outs

    R.serve_start(workers=2, max_batch=2, hbm_budget_bytes=budget)
    try:
        sids = [R.scene_register(d) for d in ds]
        round_of(sids, np.random.default_rng(61), 60)
        st = R.serve_stats()
        print(f"[serve-budget] budget {budget}, stats {st}", flush=True)
        assert st["completed"] == 60 and st["failed"] == 0
        assert st["peak_bytes"] <= budget, (st["peak_bytes"], budget)
        assert st["frame_bytes"] <= budget
    finally:
        R.serve_stop()
    # one worker, round 1 queued before it starts: every scene's frame meets a
    # two-view batch in round 1, so round 2 fits the frames it left
    R.serve_start(workers=1, max_batch=2, start_paused=True)
    try:
        sids = [R.scene_register(d) for d in ds]
        round_of(sids, np.random.default_rng(62), 60, resume=True)
        made = R.serve_stats()["frames_created"]
        assert made == len(sizes)
        round_of(sids, np.random.default_rng(63), 60)
        st = R.serve_stats()
        print(f"[serve-reuse] frames after round 1: {made}, after round 2: {st['frames_created']}; {st}", flush=True)
        assert st["frames_created"] == made
        assert st["completed"] == 120 and st["failed"] == 0
    finally:
        R.serve_stop()
