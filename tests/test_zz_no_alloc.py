"""The allocation-free forward entry point (cs_render_forward_noalloc) against
cs_render_forward: the same kernels on buffers carved from the library's static
scratch array, so every pixel must be identical (the parity bar of 1e-4 against
the oracle then carries over).  Two calls in a row, the second on a smaller
scene and image (the array keeps the first call's contents); the default HIP
memory pool's reserved and used bytes and torch's allocated bytes do not move
across the two calls; requests beyond the array's size fail with CS_ENOMEM
before any kernel runs."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_helpers import PIX_TOL, say  # noqa: E402
from paper_2411_14974_amd import scenes  # noqa: E402

_POOL_RESERVED, _POOL_USED = 0x5, 0x7  # hipMemPoolAttrReservedMemCurrent / UsedMemCurrent


def pool_bytes(device=0):
    hip = C.CDLL("libamdhip64.so")
    pool = C.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(C.byref(pool), C.c_int(device)) == 0
    out = []
    for attr in (_POOL_RESERVED, _POOL_USED):
        v = C.c_uint64()
        assert hip.hipMemPoolGetAttribute(pool, C.c_int(attr), C.byref(v)) == 0
        out.append(v.value)
    return tuple(out)


@pytest.fixture(scope="module")
def R():
    from paper_2411_14974_amd.binding import Renderer
    r = Renderer(0)
    yield r
    r.close()


def dev(scene):
    from paper_2411_14974_amd.binding import DeviceScene
    return DeviceScene.from_scene(scene, "cuda:0")


def test_noalloc_equals_plain_forward_two_calls(R):
    from paper_2411_14974_amd.binding import make_params
    big, cam_big, _ = scenes.config3()  # 1M convexes at 1920x1080
    small, cam_small, _ = scenes.config2(n=20000, width=333, height=217)
    say(f"[noalloc] scenes N={big.n} {cam_big.width}x{cam_big.height} then N={small.n} {cam_small.width}x{cam_small.height}")
    d_big, d_small = dev(big), dev(small)
    p = make_params()
    ref_big, _ = R.forward(d_big, cam_big, p)
    ref_small, _ = R.forward(d_small, cam_small, p)
    out_big = torch.full_like(ref_big, -1.0)
    out_small = torch.full_like(ref_small, -1.0)
    torch.cuda.synchronize()
    before = pool_bytes(), torch.cuda.memory_allocated()
    say("[noalloc] call 1 (1M convexes, 1080p)")
    R.forward_noalloc(d_big, cam_big, out_big, p)
    say("[noalloc] call 2 (20k convexes, 333x217)")
    R.forward_noalloc(d_small, cam_small, out_small, p)
    torch.cuda.synchronize()
    after = pool_bytes(), torch.cuda.memory_allocated()
    say(f"[noalloc] pool (reserved, used) and torch bytes before {before}, after {after}")
    assert after == before
    for name, out, ref in (("1M 1080p", out_big, ref_big), ("20k 333x217", out_small, ref_small)):
        err = float((out - ref).abs().max())
        say(f"[noalloc] {name}: max |noalloc - plain| {err:.2e}")
        assert err <= PIX_TOL
        assert torch.equal(out, ref), name
    # a third call on the first scene again: the scratch's leftovers do not leak in
    out_big.fill_(-1.0)
    R.forward_noalloc(d_big, cam_big, out_big, p)
    torch.cuda.synchronize()
    assert torch.equal(out_big, ref_big)


def test_noalloc_rejects_sizes_beyond_the_scratch(R):
    from paper_2411_14974_amd.binding import CS_ENOMEM, CSError, make_params
    small, _, _ = scenes.config2(n=100, width=64, height=64)
    d_small = dev(small)
    huge = scenes.Camera(16384, 16384, 16384.0, 16384.0, 8192.0, 8192.0)
    out = torch.empty((16384, 16384, 3), device="cuda:0")
    with pytest.raises(CSError) as ei:
        R.forward_noalloc(d_small, huge, out, make_params())
    say(f"[noalloc] 16384^2 image: {ei.value}")
    assert ei.value.code == CS_ENOMEM and "scratch" in str(ei.value)
    del out
    # 2.2M convexes need more per-convex bytes than the array holds: rejected
    # before any kernel reads the (uninitialised) arrays
    n = 2_200_000
    from paper_2411_14974_amd.binding import DeviceScene
    ds = DeviceScene(torch.empty((n, 6, 3), device="cuda:0"), torch.ones(n, device="cuda:0"),
                     torch.ones(n, device="cuda:0"), torch.full((n,), 0.5, device="cuda:0"),
                     torch.zeros((n, 16, 3), device="cuda:0"))
    cam = scenes.Camera(64, 64, 64.0, 64.0, 32.0, 32.0)
    out = torch.empty((64, 64, 3), device="cuda:0")
    with pytest.raises(CSError) as ei:
        R.forward_noalloc(ds, cam, out, make_params())
    say(f"[noalloc] {n} convexes: {ei.value}")
    assert ei.value.code == CS_ENOMEM
