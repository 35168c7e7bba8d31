"""The C-ABI library: it loads, exports every symbol the header declares, and
returns its documented error codes on bad arguments (no compute call is made,
so these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2411_14974_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "convexsplat.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(cs_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for s in ("cs_create", "cs_destroy", "cs_render_forward", "cs_render_backward", "cs_state_release",
              "cs_debug_preprocess", "cs_last_error"):
        assert s in syms
    assert set(syms) == set(binding.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert L.cs_version() >= 100


def test_null_and_shape_errors_without_a_gpu():
    L = binding.lib()
    cam = binding.Camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.znear = 64, 64, 50.0, 50.0, 0.1
    sc = binding.SceneS(10, 6, 3, 0, 0, 0, 0, 0)
    out = C.c_void_p()
    # NULL context
    assert L.cs_render_forward(None, C.byref(sc), C.byref(cam), None, 1, None, None) == binding.CS_EINVAL
    assert b"ctx" in L.cs_last_error()
    # a context-sized dummy: argument checks run before any device call
    dummy = (C.c_char * 64)()
    bad_k = binding.SceneS(10, 9, 3, 1, 1, 1, 1, 1)
    assert L.cs_render_forward(dummy, C.byref(bad_k), C.byref(cam), None, 1, None, None) == binding.CS_EINVAL
    assert b"k" in L.cs_last_error()
    bad_deg = binding.SceneS(10, 6, 4, 1, 1, 1, 1, 1)
    assert L.cs_render_forward(dummy, C.byref(bad_deg), C.byref(cam), None, 1, None, None) == binding.CS_EINVAL
    null_arr = binding.SceneS(10, 6, 3, 1, 0, 1, 1, 1)
    assert L.cs_render_forward(dummy, C.byref(null_arr), C.byref(cam), None, 1, None, None) == binding.CS_EINVAL
    bad_cam = binding.Camera()
    bad_cam.width, bad_cam.height, bad_cam.fx, bad_cam.fy, bad_cam.znear = 0, 64, 50.0, 50.0, 0.1
    good = binding.SceneS(10, 6, 3, 1, 1, 1, 1, 1)
    assert L.cs_render_forward(dummy, C.byref(good), C.byref(bad_cam), None, 1, None, None) == binding.CS_EINVAL
    p = binding.make_params(tile=12)
    assert L.cs_render_forward(dummy, C.byref(good), C.byref(cam), C.byref(p), 1, None, None) == binding.CS_EINVAL
    p = binding.make_params(flags=binding.FLAG_DIGITS(3))
    assert L.cs_render_forward(dummy, C.byref(good), C.byref(cam), C.byref(p), 1, None, None) == binding.CS_EINVAL
    # batched: view count and output pointers are checked first
    cams = (binding.Camera * 2)(cam, cam)
    outs = (C.c_void_p * 2)(1, 1)
    assert L.cs_render_forward_batch(dummy, C.byref(good), 0, cams, None, outs, None, None) == binding.CS_EINVAL
    null_outs = (C.c_void_p * 2)(1, 0)
    assert L.cs_render_forward_batch(dummy, C.byref(good), 2, cams, None, null_outs, None, None) == binding.CS_EINVAL
    assert L.cs_batch_check(None, None) == binding.CS_EINVAL
    assert L.cs_render_backward(dummy, C.byref(good), C.byref(cam), None, None, 1, 1, None) == binding.CS_EINVAL


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"),
                    reason="a GPU is present: cs_create would succeed")
def test_create_without_device_reports_enodev():
    L = binding.lib()
    h = C.c_void_p()
    rc = L.cs_create(0, 0, C.byref(h))
    assert rc == binding.CS_ENODEV
    assert not h.value


def test_bad_scene_dtype_is_rejected():
    L = binding.lib()
    cam = binding.Camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.znear = 64, 64, 50.0, 50.0, 0.1
    dummy = (C.c_char * 64)()
    bad = binding.SceneS(10, 6, 3, 1, 1, 1, 1, 1, 3)
    assert L.cs_render_forward(dummy, C.byref(bad), C.byref(cam), None, 1, None, None) == binding.CS_EINVAL
    assert b"dtype" in L.cs_last_error()


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the C compiler's sizes and offsets
    for the header's structs (a C probe compiled with gcc prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"cs_scene": binding.SceneS, "cs_camera": binding.Camera, "cs_grads": binding.GradsS,
               "cs_params": binding.Params, "cs_serve_config": binding.ServeConfig,
               "cs_serve_stats": binding.ServeStats, "cs_tuning": binding.Tuning,
               "cs_debug_convex": binding.DebugConvex}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "convexsplat.h"', "int main(void) {"]
    for name, S in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in S._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, v = ln.split()
        got[(name, field)] = int(v)
    for name, S in structs.items():
        assert got[(name, "size")] == C.sizeof(S), name
        for f, _ in S._fields_:
            assert got[(name, f)] == getattr(S, f).offset, (name, f)


def test_training_entry_points_reject_bad_arguments_without_a_gpu():
    """Argument checks of the density-control, loss, optimiser and
    initialisation entry points run before any device call."""
    L = binding.lib()
    dummy = (C.c_char * 64)()
    E = binding.CS_EINVAL
    sc = binding.SceneS(10, 6, 3, 1, 1, 1, 1, 1)
    dp = binding.make_densify_params()
    out = binding.SceneOut(1, 1, 1, 1, 1, 1)
    n_out = C.c_int64()
    assert L.cs_densify(None, C.byref(sc), 1, 1, C.byref(dp), 10, C.byref(out), C.byref(n_out), None) == E
    assert L.cs_densify(dummy, C.byref(sc), None, 1, C.byref(dp), 10, C.byref(out), C.byref(n_out), None) == E
    assert L.cs_densify(dummy, C.byref(sc), 1, 1, None, 10, C.byref(out), C.byref(n_out), None) == E
    assert L.cs_densify(dummy, C.byref(sc), 1, 1, C.byref(dp), -1, C.byref(out), C.byref(n_out), None) == E
    half = binding.SceneS(10, 6, 3, 1, 1, 1, 1, 1, binding.DTYPE_F16)
    assert L.cs_densify(dummy, C.byref(half), 1, 1, C.byref(dp), 10, C.byref(out), C.byref(n_out), None) == E
    assert b"float32" in L.cs_last_error()
    assert L.cs_densify_accumulate(dummy, None, 1, 1, 1, None) == E
    # loss: null pointers, bad size, lambda outside [0, 1]
    assert L.cs_ssim_loss_grad(dummy, None, 1, 8, 8, 0.2, 1, 1, None) == E
    assert L.cs_ssim_loss_grad(dummy, 1, 1, 0, 8, 0.2, 1, 1, None) == E
    assert L.cs_ssim_loss_grad(dummy, 1, 1, 8, 8, 1.5, 1, 1, None) == E
    # Adam: step 0, betas outside [0, 1), bad K
    g = binding.GradsS(1, 1, 1, 1, 1)
    ps = binding.ParamSet(1, 1, 1, 1, 1)
    ap = binding.make_adam_params(0)
    assert L.cs_adam_step(dummy, 10, 6, 3, C.byref(g), C.byref(ps), C.byref(ps), C.byref(ps), None, C.byref(ap),
                          None) == E
    ap = binding.make_adam_params(1, beta2=1.0)
    assert L.cs_adam_step(dummy, 10, 6, 3, C.byref(g), C.byref(ps), C.byref(ps), C.byref(ps), None, C.byref(ap),
                          None) == E
    ap = binding.make_adam_params(1)
    assert L.cs_adam_step(dummy, 10, 9, 3, C.byref(g), C.byref(ps), C.byref(ps), C.byref(ps), None, C.byref(ap),
                          None) == E
    # initialisation: bad K, missing output
    ip = binding.make_init_params()
    assert L.cs_init_from_points(dummy, 10, 1, None, 2, 3, C.byref(ip), C.byref(ps), None) == E
    assert L.cs_init_from_points(dummy, 10, 1, None, 6, 3, C.byref(ip), None, None) == E
