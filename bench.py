#!/usr/bin/env python3
"""Benchmark of the smooth-convex rasterizer on one MI355X.

A step is one training pass of the whole hot path over one synthetic view:
forward render (preprocess, depth sort, binning, tile sort, ranges, per-tile
compositing), the L1 loss gradient, and the backward render (per-tile reverse
compositing, per-convex chain rule) to gradients for points, delta, sigma,
opacity and SH.  Inputs are resident in HBM before the timed region.

Default workload: 1M convexes (K=6, SH degree 3, 64-component mixture) at
1920x1080, the paper-scale scene.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12 lane-operations/s for
# full-rate ops (FP32 and FP64 FMA alike on this chip); a transcendental costs TRANS_SLOTS.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def workload(name):
    from paper_2411_14974_amd import scenes
    if name == "c3":
        scene, cam, target = scenes.config3()
        desc = "1M convexes K=6 SH3, 64-cluster mixture, 1920x1080, fwd+bwd (L1)"
    elif name == "c2":
        scene, cam, target = scenes.config2()
        desc = "100k convexes K=6 SH3, uniform cube, 1297x840, fwd+bwd (L1)"
    else:
        raise SystemExit(f"unknown workload {name}")
    return scene, cam, target, desc


# Issue slots of one float32 transcendental (v_exp_f32, v_log_f32, v_rcp_f32) in
# full-rate VALU operations: measured on the MI355X with chains of exp2 against
# chains of FMA (half rate), where an earlier estimate assumed quarter rate.
TRANS_SLOTS = 2


def pair_cost(stage, T):
    """VALU lane-operations of one full (pixel, convex) pair evaluation with T
    hull lines, a transcendental counted as TRANS_SLOTS full-rate operations:
    forward (T + 3) transcendentals, 2T FP64 FMA, 3T + 12 FP32 operations;
    backward (T + 4) transcendentals, 2T FP64 FMA, 12T + 30 FP32 operations."""
    if stage == "render_fwd":
        return TRANS_SLOTS * (T + 3) + 2 * T + (3 * T + 12)
    return TRANS_SLOTS * (T + 4) + 2 * T + (12 * T + 30)


def stage_work(stage, n, m, K, deg, cnt):
    """Algorithmic bytes (or VALU lane-operations) of one launch of a stage;
    cnt: the device work counters of the step (cs_state_counters)."""
    nc = (deg + 1) ** 2
    T_mean = cnt["sum_T_full"] / max(cnt["full_bwd"], 1)
    rec = 48 + 24 * T_mean  # header + the T hull lines written
    if stage == "preprocess":  # read points, delta, sigma, opacity, SH; write record, key, id, binning record, hull
        return "hbm", n * (12 * K + 12 + 12 * nc + rec + 4 + 4 + 16 + 4)
    if stage == "depth_sort":  # one histogram read (4 B) + 4 passes x (read 8 B + write 8 B)
        return "hbm", n * (4 + 4 * 16)
    if stage == "bin_scan":  # read id 4 + binning record 16; write it in depth order 16 + count 4 + offset 4
        return "hbm", n * 44
    if stage == "emit":  # per convex: id, offset, binning record 24 B; per pair: write 8 B
        return "hbm", n * 24 + m * 8
    if stage == "tile_sort":  # one histogram read (4 B) + 2 passes x (read 8 B + write 8 B) over the pairs
        return "hbm", m * (4 + 2 * 16)
    if stage == "ranges":
        return "hbm", m * 4
    if stage == "render_fwd":  # full pairs x the forward per-pair cost at the measured mean hull size
        return "alu", cnt["full"] * pair_cost(stage, T_mean)
    if stage == "render_bwd":
        return "alu", cnt["full_bwd"] * pair_cost(stage, T_mean)
    if stage == "preprocess_bwd":  # read accumulators, points, delta, sigma, SH, hull; write gradients
        acc = 4 * (3 * K + 6)
        return "hbm", n * (acc + 12 * K + 8 + 12 * nc + 4 + 12 * K + 12 + 12 * nc)
    return "hbm", 0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_batched(steps, warmup):
    """32 views of the 500k-convex mixture scene, fwd+bwd: batched graph vs plain per-view loop."""
    import torch

    from paper_2411_14974_amd import scenes
    from paper_2411_14974_amd.binding import (FLAG_AUTOTUNE, FLAG_GRAPH, FLAG_TIMING, DeviceScene, Renderer,
                                              make_params)
    scene, cams, targets = scenes.config4()
    dev = torch.device("cuda:0")
    R = Renderer(0)
    ds = DeviceScene.from_scene(scene, dev)
    tg = [torch.from_numpy(t).to(dev) for t in targets]
    outs = [torch.empty_like(t) for t in tg]
    dls = [torch.empty_like(t) for t in tg]
    grads = {k: torch.empty_like(getattr(ds, k)) for k in ("points", "delta", "sigma", "opacity", "sh")}
    mpix = sum(c.width * c.height for c in cams) / 1e6
    t0 = time.perf_counter()
    tune = R.autotune(ds, cams)
    tune_s = time.perf_counter() - t0
    pb = make_params(flags=FLAG_GRAPH | FLAG_AUTOTUNE)

    def batched():
        o, st = R.forward_batch(ds, cams, pb, want_state=True, outs=outs)
        for a, t, d in zip(o, tg, dls):
            R.l1_loss_grad(a, t, grad=d)
        R.backward_batch(st, dls, grads=grads)
        return st

    pp = make_params()

    def plain():
        for c, a, t, d in zip(cams, outs, tg, dls):
            o, st = R.forward(ds, c, pp, want_state=True, out=a)
            R.l1_loss_grad(o, t, grad=d)
            R.backward(st, d, grads=grads)
            st.release()

    res = {}
    for name, fn in (("batched", batched), ("plain", plain)):
        for _ in range(warmup):
            r = fn()
            if r is not None:
                r.release()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        keep = []
        for _ in range(steps):
            r = fn()
            if r is not None:
                keep.append(r)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        for r in keep:
            r.release()
        res[name] = {"ms_per_step": ms, "mpixels_per_s": mpix / (ms / 1e3)}
    R.close()
    return {
        "workload": "500k convexes K=6 SH3 mixture, 32 views (960x540 / 1297x840 / 1920x1080), fwd+bwd (L1)",
        "mpixels_per_batch": mpix,
        "batched_graph": res["batched"],
        "plain_per_view": res["plain"],
        "speedup": res["plain"]["ms_per_step"] / res["batched"]["ms_per_step"],
        "autotune": {**tune, "seconds": tune_s},
    }


def window_mean(st0, st1, key):
    """Mean of a per-request server statistic over the requests finished
    between two snapshots (the server reports running means)."""
    n0 = st0["completed"] + st0["failed"]
    n1 = st1["completed"] + st1["failed"]
    return (st1[key] * n1 - st0[key] * n0) / max(n1 - n0, 1)


def bench_serving(rates, duration, max_batch=4, workers=2):
    """Poisson request streams against 4 resident scenes (0.2/0.5/1/2 M convexes), forward only:
    continuous batching (worker streams taking batches of one scene's queued requests) vs plain FIFO one
    request at a time."""
    import torch

    from paper_2411_14974_amd import scenes
    from paper_2411_14974_amd.binding import DeviceScene, Renderer, make_camera
    dev = torch.device("cuda:0")
    ds = [DeviceScene.from_scene(scenes.serve_scene(i), dev) for i in range(4)]
    R = Renderer(0)
    pools = {wh: [torch.empty((wh[1], wh[0], 3), device=dev) for _ in range(48)] for wh in scenes.RESOLUTIONS_C5}
    out = {"workload": "4 resident mixture scenes of 0.2/0.5/1/2 M convexes (K=6, SH3); requests uniform over "
                       "scenes and 256x256 / 960x540 / 1920x1080, random orbit poses, Poisson arrivals, forward only",
           "duration_s_per_rate": duration, "continuous_batching": {"workers": workers, "max_batch": max_batch},
           "modes": {}}
    for mode, cfg in (("continuous_batching", dict(workers=workers, max_batch=max_batch)),
                      ("plain_fifo", dict(workers=1, max_batch=1))):
        R.serve_start(hbm_budget_bytes=96 << 30, **cfg)
        sids = [R.scene_register(d) for d in ds]
        # warm-up: half a second of the highest rate's request mix (other poses), so
        # that the workers' frames and the memory pool have met every scene,
        # resolution and batch size before the measured streams
        warm = scenes.serve_requests(max(rates), 0.5, variant=9)
        t0, wid = time.perf_counter(), []
        for k, (ta, s_, c) in enumerate(warm):
            while ta > time.perf_counter() - t0:
                time.sleep(2e-4)
            rc, rid = R.serve_submit_raw(sids[s_], make_camera(c), pools[(c.width, c.height)][k % 48].data_ptr())
            if rc == 0:
                wid.append(rid)
        for r_ in wid:
            R.serve_wait(r_)
        rows = []
        for rate in rates:
            reqs = [(t, sids[s], make_camera(c)) for t, s, c in scenes.serve_requests(rate, duration)]
            st0 = R.serve_stats()
            ids, pix, k = [], 0, 0
            t0 = time.perf_counter()
            for ta, sid, cam in reqs:
                while True:
                    dt = ta - (time.perf_counter() - t0)
                    if dt <= 0:
                        break
                    time.sleep(min(dt, 2e-4))
                buf = pools[(cam.width, cam.height)][k % 48]
                k += 1
                rc, rid = R.serve_submit_raw(sid, cam, buf.data_ptr())
                if rc == 0:
                    ids.append(rid)
                    pix += cam.width * cam.height
            lat = np.array([R.serve_wait(r) for r in ids])
            wall = time.perf_counter() - t0
            st = R.serve_stats()
            nb = st["batches"] - st0["batches"]
            nr = (st["completed"] + st["failed"]) - (st0["completed"] + st0["failed"])
            rows.append({"rate_rps": rate, "requests": len(ids), "p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)), "mpixels_per_s": pix / wall / 1e6,
                         "mean_batch": nr / nb if nb else 0.0,
                         "frames_created": st["frames_created"] - st0["frames_created"],
                         "mean_queue_ms": window_mean(st0, st, "mean_queue_ms"),
                         "mean_run_ms": window_mean(st0, st, "mean_run_ms"),
                         "frame_gb": st["frame_bytes"] / 1e9})
            print(f"[serve] {mode} {rate:g} req/s: {len(ids)} requests, p99 {rows[-1]['p99_ms']:.2f} ms",
                  file=sys.stderr, flush=True)
        R.serve_stop()
        out["modes"][mode] = rows
    R.close()
    return out


def bench_light(scene, cam, target, steps, warmup, ms_f32):
    """The same fwd+bwd step with the scene stored in 16-bit floats (the paper's
    light model, Sec. 4.2): IEEE half storage, float32 arithmetic, float32 gradients."""
    import torch

    from paper_2411_14974_amd.binding import FLAG_TIMING, DeviceScene, Renderer, make_params
    dev = torch.device("cuda:0")
    R = Renderer(0)
    ds = DeviceScene.from_scene(scene, dev, dtype=torch.float16)
    tgt = torch.from_numpy(target).to(dev)
    H, W = tgt.shape[:2]
    rgb = torch.empty((H, W, 3), device=dev)
    dl = torch.empty_like(rgb)
    grads = {k: torch.empty_like(getattr(ds, k), dtype=torch.float32) for k in ("points", "delta", "sigma", "opacity", "sh")}

    def step(params):
        out, st = R.forward(ds, cam, params, want_state=True, out=rgb)
        R.l1_loss_grad(out, tgt, grad=dl)
        R.backward(st, dl, grads=grads)
        return st

    def run(params, n):
        held = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            held.append(step(params))
            if len(held) > 2:
                held.pop(0).release()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for s in held:
            s.release()
        return (t1 - t0) * 1e3 / n

    run(make_params(), max(warmup, 3))
    ms = run(make_params(), steps)
    R.timing(reset=True)
    run(make_params(flags=FLAG_TIMING), steps)
    tm = R.timing(reset=True)
    R.close()
    scene_bytes = sum(getattr(ds, k).numel() * 2 for k in ("points", "delta", "sigma", "opacity", "sh"))
    return {"storage": "float16 scene arrays, float32 arithmetic and gradients", "ms_per_step": ms,
            "mpixels_per_s": W * H / (ms / 1e3) / 1e6, "speedup_vs_f32": ms_f32 / ms,
            "scene_mb": scene_bytes / 1e6,
            "stages_ms": {k: round(t / c, 4) for k, (t, c) in tm.items() if c and k.startswith("preprocess")}}


def bench_train(scene, cam, target, steps, warmup):
    """A full training step of the paper's optimisation (Sec. 3.3): render,
    (1 - 0.2) L1 + 0.2 D-SSIM loss and its gradient, backward, fused Adam on
    the raw parameters writing the next step's activated scene."""
    import torch

    from paper_2411_14974_amd.binding import PARAM_NAMES, DeviceScene, Renderer, make_adam_params, make_params
    dev = torch.device("cuda:0")
    R = Renderer(0)
    act = DeviceScene.from_scene(scene, dev)
    raw = {"points": act.points.clone(), "delta": torch.log(act.delta), "sigma": torch.log(act.sigma),
           "opacity": torch.logit(act.opacity), "sh": act.sh.clone()}
    actd = {k: getattr(act, k) for k in PARAM_NAMES}
    m = {k: torch.zeros_like(v) for k, v in raw.items()}
    v2 = {k: torch.zeros_like(v) for k, v in raw.items()}
    grads = {k: torch.empty_like(v) for k, v in raw.items()}
    tgt = torch.from_numpy(target).to(dev)
    H, W = tgt.shape[:2]
    rgb = torch.empty((H, W, 3), device=dev)
    dl = torch.empty_like(rgb)
    loss = torch.zeros(1, device=dev)
    params = make_params()

    def step(t):
        out, st = R.forward(act, cam, params, want_state=True, out=rgb)
        R.ssim_loss_grad(out, tgt, 0.2, grad=dl, loss=loss)
        R.backward(st, dl, grads=grads)
        R.adam_step(grads, raw, m, v2, actd, make_adam_params(t))
        return st

    held, t = [], 1
    for _ in range(max(warmup, 3)):
        held.append(step(t))
        t += 1
        if len(held) > 2:
            held.pop(0).release()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        held.append(step(t))
        t += 1
        if len(held) > 2:
            held.pop(0).release()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    for s_ in held:
        s_.release()
    R.close()
    return {"step": "render + L1/D-SSIM loss + backward + Adam (raw parameters, activations fused)",
            "ms_per_step": ms, "mpixels_per_s": W * H / (ms / 1e3) / 1e6}


def bench_densify(scene, steps):
    """One split / prune step (paper Sec. 3.3) over the workload's scene: 5 % of
    the convexes split, those below opacity 0.03 pruned (about 2.5 % of this
    scene), the size limit at the radius distribution's upper tail."""
    import torch

    from paper_2411_14974_amd.binding import DeviceScene, Renderer, make_densify_params
    dev = torch.device("cuda:0")
    R = Renderer(0)
    ds = DeviceScene.from_scene(scene, dev)
    rng = np.random.default_rng(77)
    n = scene.n
    denom = torch.from_numpy(rng.integers(1, 4, n).astype(np.float32)).to(dev)
    mean = np.where(rng.random(n) < 0.05, 1e-5, 1e-6).astype(np.float32)
    accum = denom * torch.from_numpy(mean).to(dev)
    p = make_densify_params(size_max=0.2)
    cap = 2 * n
    out, src = R.densify(ds, accum, denom, p, capacity=cap)  # warm-up, sizes the outputs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out, src = R.densify(ds, accum, denom, p, capacity=cap)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    row = 4 * (3 * scene.k + 3 + 3 * (scene.deg + 1) ** 2)
    moved = n * (2 * row + 8) + out.n * (row + 4)  # read (classify + scatter) + statistic; write outputs
    R.close()
    return {"workload": f"split/prune of the {n}-convex scene", "convexes_out": out.n, "ms": ms,
            "gb_per_s": moved / (ms / 1e3) / 1e9,
            "note": "host-timed call, including the 8-byte count read-back and the binding's output allocation"}


def counter_traffic(stage, workload):
    """HBM bytes per launch of a stage's kernel from the committed rocprofv3
    counters (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by what the same
    counters read for a device copy of known size), or None when there are none
    for this workload or the kernel's source has changed since they were taken."""
    if workload != "c3":
        return None
    path = os.path.join(ROOT, "profiles", "counters_c3_1M_1080p.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    for name, k in d["kernels"].items():
        if name.startswith(stage + "_kernel"):
            with open(os.path.join(ROOT, k["source"]), "rb") as f:
                if hashlib.sha1(f.read()).hexdigest() != k["source_sha1"]:
                    return None
            return (k["fetch_kib"] * d["fetch_scale"] + k["write_kib"] * d["write_scale"]) * 1024.0
    return None


def bench_small_configs(steps, warmup, with_oracle):
    """The two smaller workloads: 1k convexes at 128x128, forward only, and
    100k convexes at 1297x840, forward + L1 backward; GPU Mpixels/s of the plain
    renderer, and the FP64 oracle's Mpixels/s over the whole frame (1k:
    forward; 100k: forward and backward)."""
    import torch

    from paper_2411_14974_amd import scenes
    from paper_2411_14974_amd.binding import DeviceScene, Renderer, make_params
    dev = torch.device("cuda:0")
    R = Renderer(0)
    out = {}
    for name in ("c1", "c2"):
        if name == "c1":
            scene, cam = scenes.config1()
            target = None
        else:
            scene, cam, target = scenes.config2()
        W, H = cam.width, cam.height
        ds = DeviceScene.from_scene(scene, dev)
        rgb = torch.empty((H, W, 3), device=dev)
        dl = torch.empty_like(rgb)
        tgt = torch.from_numpy(target).to(dev) if target is not None else None
        grads = {k: torch.empty_like(getattr(ds, k)) for k in ("points", "delta", "sigma", "opacity", "sh")}

        def step():
            if tgt is None:
                R.forward(ds, cam, make_params(), out=rgb)
                return None
            o, st = R.forward(ds, cam, make_params(), want_state=True, out=rgb)
            R.l1_loss_grad(o, tgt, grad=dl)
            R.backward(st, dl, grads=grads)
            return st

        def run(k):
            held = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                held.append(step())
                if len(held) > 2 and held[0] is not None:
                    held.pop(0).release()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for s_ in held:
                if s_ is not None:
                    s_.release()
            return (t1 - t0) * 1e3 / k

        run(max(warmup, 3))
        ms = run(steps)
        d = {"workload": ("1k convexes K=6 SH0, 128x128, forward only" if name == "c1"
                          else "100k convexes K=6 SH3, 1297x840, fwd+bwd (L1)"),
             "ms_per_step": ms, "mpixels_per_s": W * H / (ms / 1e3) / 1e6}
        if with_oracle:
            import oracle
            if name == "c1":
                t0 = time.perf_counter()
                oracle.render(scene, cam, mode=oracle.MODE_MATCHED)
                d["oracle_mpixels_per_s"] = W * H / (time.perf_counter() - t0) / 1e6
                d["oracle_sample"] = "whole frame, forward"
            else:
                cb = cpu_baseline(scene, cam, target, W * H)
                d["oracle_mpixels_per_s"] = cb["value"]
                d["oracle_sample"] = cb["sample"]
        out[name] = d
    R.close()
    return out


def cpu_baseline(scene, cam, target, sample):
    """The FP64 oracle, as it stands, on a seeded pixel sample of the workload."""
    import oracle
    W, H = cam.width, cam.height
    whole = sample >= W * H
    if whole:
        pix, sel = None, np.arange(W * H)
    else:
        rng = np.random.default_rng(2024)
        sel = rng.choice(W * H, sample, replace=False)
        pix = np.stack([sel % W, sel // W], 1).astype(np.int32)
    t0 = time.perf_counter()
    oracle.preprocess(scene, cam)
    t_pre = time.perf_counter() - t0
    t0 = time.perf_counter()
    rgb, _, _ = oracle.render(scene, cam, mode=oracle.MODE_MATCHED, pixels=pix)
    t_fwd = time.perf_counter() - t0
    dl = np.sign(rgb.reshape(-1, 3) - target.reshape(-1, 3)[sel]) / (3.0 * W * H)
    t0 = time.perf_counter()
    oracle.backward(scene, cam, dl, mode=oracle.MODE_MATCHED, pixels=pix)
    t_bwd = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if whole:
        return {"value": W * H / (t_fwd + t_bwd) / 1e6, "unit": "Mpixels/s", "cores": cores, "kind": "oracle",
                "cpu": cpu_model(),
                "sample": f"the whole frame, fwd+bwd, matched mode; measured {t_fwd + t_bwd:.1f} s of CPU work"}
    # each oracle call runs its own per-convex preprocess once; the rest scales with pixels
    per_pixel = max(t_fwd + t_bwd - 2 * t_pre, 1e-12) / sample
    full = 2 * t_pre + W * H * per_pixel
    return {
        "value": W * H / full / 1e6, "unit": "Mpixels/s", "cores": cores, "kind": "oracle", "cpu": cpu_model(),
        "sample": (f"{sample} seeded pixels of the same frame, fwd+bwd, matched mode; full-frame time "
                   f"extrapolated as 2 x per-convex pass ({t_pre:.2f} s) + W*H x per-pixel cost "
                   f"({per_pixel * 1e3:.3f} ms); measured {t_pre + t_fwd + t_bwd:.1f} s of CPU work"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--cpu-sample", type=int, default=163840)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stages", action="store_true", help="print per-stage times to stderr")
    ap.add_argument("--forms", default="plain,configs,light,train,densify,batched,serving",
                    help="comma list of plain, configs (the 1k and 100k workloads), light (16-bit scene), train, "
                         "densify, batched, serving")
    ap.add_argument("--serve-rates", default="50,100,200,500,1000,2000,4000",
                    help="request rates (req/s) of the serving sweep (4000: beyond both modes' capacity)")
    ap.add_argument("--serve-seconds", type=float, default=8.0)
    ap.add_argument("--serve-max-batch", type=int, default=4, help="requests per batch of continuous batching")
    ap.add_argument("--serve-workers", type=int, default=2, help="worker streams of continuous batching")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (views shard across GPUs with no "
              "exchange; see the sharding design). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2411_14974_amd.binding import FLAG_TIMING, DeviceScene, Renderer, make_params

    scene, cam, target, desc = workload(args.workload)
    W, H = cam.width, cam.height
    dev = torch.device("cuda:0")
    R = Renderer(0)
    ds = DeviceScene.from_scene(scene, dev)
    tgt = torch.from_numpy(target).to(dev)
    rgb = torch.empty((H, W, 3), device=dev)
    dl = torch.empty_like(rgb)
    grads = {k: torch.empty_like(getattr(ds, k)) for k in ("points", "delta", "sigma", "opacity", "sh")}
    plain_params, timed_params = make_params(), make_params(flags=FLAG_TIMING)

    def step(params):
        out, st = R.forward(ds, cam, params, want_state=True, out=rgb)
        R.l1_loss_grad(out, tgt, grad=dl)
        R.backward(st, dl, grads=grads)
        return st

    def run(params):
        """Exactly args.steps steps between two synchronisations; per-step HIP
        events on the call stream give the step-time distribution."""
        states = []
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for i in range(args.steps):
            states.append(step(params))
            ev[i + 1].record()
            if len(states) > 2:
                states.pop(0).release()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cnt = states[-1].counters()
        for s in states:
            s.release()
        per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
        return (t1 - t0) * 1e3 / args.steps, cnt, per

    # warm-up in the timed loop's pattern (two states held), so that the
    # context's frame cache reaches its steady state before timing
    held = []
    for _ in range(max(args.warmup, 3)):
        held.append(step(plain_params))
        if len(held) > 2:
            held.pop(0).release()
    for s in held:
        s.release()
    # the step time: no stage events in the stream
    ms, cnt, per_step = run(plain_params)
    # per-stage kernel times: the same steps again, with HIP events around each stage
    R.timing(reset=True)
    ms_timed, _, _ = run(timed_params)
    timing = R.timing(reset=True)

    n, K, deg = scene.n, scene.k, scene.deg
    avg = {s: (t / c if c else 0.0) for s, (t, c) in timing.items()}
    dom = max(avg, key=avg.get)
    bound, work = stage_work(dom, n, cnt["pairs"], K, deg, cnt)
    sec = avg[dom] / 1e3
    if bound == "hbm":
        achieved, peak, unit = work / sec / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = work / sec / 1e12, VALU_PEAK_TOPS, "TOP/s"
    if args.stages:
        for s in avg:
            print(f"  {s:15s} {avg[s]:8.3f} ms", file=sys.stderr)
        print(f"  counters {cnt}", file=sys.stderr)
    work_counts = {
        "pairs": cnt["pairs"], "tested": cnt["tested"], "full": cnt["full"], "full_bwd": cnt["full_bwd"],
        "T_mean": cnt["sum_T_full"] / max(cnt["full_bwd"], 1),
        "wave_evals": cnt["wave_evals"],
        "lane_utilisation": cnt["full_bwd"] / max(64 * cnt["wave_evals"], 1),
    }

    line = {
        "metric": "Mpixels/s fwd+bwd @1M convexes 1080p vs plain; p50/p99 served frame latency",
        "value": W * H / (ms / 1e3) / 1e6,
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "convexes": n, "k": K, "sh_degree": deg, "width": W, "height": H,
                   "form": "plain (one view per launch)", "tile": 16},
        "step_ms": {"p10": float(np.percentile(per_step, 10)), "p50": float(np.median(per_step)),
                    "p90": float(np.percentile(per_step, 90)), "steps": int(per_step.size)},
        "stages_ms": {s: round(v, 4) for s, v in avg.items()},
        "ms_per_step_with_stage_events": ms_timed,
        "work": work_counts,
        "roofline": {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": counter_traffic(dom, args.workload)},
    }
    if args.copy_calibration:
        a = torch.ones(64 << 20, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    R.close()
    forms = set(args.forms.split(","))
    if "configs" in forms:
        line["other_configs"] = bench_small_configs(args.steps, args.warmup, not args.no_cpu_baseline)
    if "light" in forms:
        line["light_16bit"] = bench_light(scene, cam, target, args.steps, args.warmup, ms)
    if "train" in forms:
        line["train_step"] = bench_train(scene, cam, target, args.steps, args.warmup)
    if "densify" in forms:
        line["densify"] = bench_densify(scene, args.steps)
    if "batched" in forms:
        line["batched"] = bench_batched(max(3, args.steps // 4), 2)
    if "serving" in forms:
        line["serving"] = bench_serving([float(r) for r in args.serve_rates.split(",")], args.serve_seconds,
                                        args.serve_max_batch, args.serve_workers)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(scene, cam, target, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
