"""The fused Adam step (paper Sec. 3.3: sigmoid opacity, exponential delta and
sigma, Adam on the raw parameters) against torch.optim.Adam in float64 on the
CPU, with the activations' chain rule taken by torch autograd.  Bar: raw
parameters, moments and activated outputs within 1e-5 relative (float32
arithmetic against float64) after three steps with changing gradients."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

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


def activations(raw):
    return {"points": raw["points"], "delta": torch.exp(raw["delta"]), "sigma": torch.exp(raw["sigma"]),
            "opacity": torch.sigmoid(raw["opacity"]), "sh": raw["sh"]}


@pytest.mark.parametrize("n,k,deg", [(5000, 6, 3), (777, 4, 1), (33, 8, 0)])
def test_adam_step_matches_torch(R, n, k, deg):
    from paper_2411_14974_amd.binding import make_adam_params
    rng = np.random.default_rng(n + k)
    nc = (deg + 1) ** 2
    shapes = {"points": (n, k, 3), "delta": (n,), "sigma": (n,), "opacity": (n,), "sh": (n, nc, 3)}
    raw0 = {kk: rng.normal(0, 1, s) for kk, s in shapes.items()}
    # reference: float64 parameters, one group per rate, like the kernel's
    ref = {kk: torch.tensor(raw0[kk], dtype=torch.float64, requires_grad=True) for kk in NAMES}
    ref_dc = torch.tensor(raw0["sh"][:, :1], dtype=torch.float64, requires_grad=True)
    ref_rest = torch.tensor(raw0["sh"][:, 1:], dtype=torch.float64, requires_grad=True)
    lrs = dict(lr_points=1e-3, lr_delta=0.005, lr_sigma=0.0045, lr_opacity=0.05, lr_sh_dc=0.0025, lr_sh_rest=1e-4)
    opt = torch.optim.Adam([{"params": [ref["points"]], "lr": lrs["lr_points"]},
                            {"params": [ref["delta"]], "lr": lrs["lr_delta"]},
                            {"params": [ref["sigma"]], "lr": lrs["lr_sigma"]},
                            {"params": [ref["opacity"]], "lr": lrs["lr_opacity"]},
                            {"params": [ref_dc], "lr": lrs["lr_sh_dc"]},
                            {"params": [ref_rest], "lr": lrs["lr_sh_rest"]}], betas=(0.9, 0.999), eps=1e-8)
    dev = {kk: torch.tensor(raw0[kk], dtype=torch.float32, device="cuda") for kk in NAMES}
    m = {kk: torch.zeros_like(dev[kk]) for kk in NAMES}
    v = {kk: torch.zeros_like(dev[kk]) for kk in NAMES}
    act = {kk: torch.empty_like(dev[kk]) for kk in NAMES}
    for step in (1, 2, 3):
        g_act = {kk: rng.normal(0, 10.0 ** rng.integers(-6, 0), s).astype(np.float32) for kk, s in shapes.items()}
        if step == 2:
            g_act["delta"][: n // 3] = 0.0  # zero gradients: m, v decay, no nan
        # reference gradients of the raw parameters through the activations
        opt.zero_grad()
        sh_full = torch.cat([ref_dc, ref_rest], dim=1)
        a = activations({"points": ref["points"], "delta": ref["delta"], "sigma": ref["sigma"],
                         "opacity": ref["opacity"], "sh": sh_full})
        loss = sum((a[kk] * torch.tensor(g_act[kk].astype(np.float64))).sum() for kk in NAMES)
        loss.backward()
        opt.step()
        grads = {kk: torch.from_numpy(g_act[kk]).cuda() for kk in NAMES}
        R.adam_step(grads, dev, m, v, act, make_adam_params(step, eps=1e-8, **lrs))
        torch.cuda.synchronize()
        want = {"points": ref["points"], "delta": ref["delta"], "sigma": ref["sigma"], "opacity": ref["opacity"],
                "sh": torch.cat([ref_dc, ref_rest], dim=1)}
        for kk in NAMES:
            got = dev[kk].cpu().double()
            exp = want[kk].detach()
            err = float(((got - exp).abs() / (exp.abs() + 1e-3)).max())
            assert err <= 1e-5, (step, kk, err)
        wa = activations({kk: want[kk].detach() for kk in NAMES})
        for kk in NAMES:
            got = act[kk].cpu().double()
            err = float(((got - wa[kk]).abs() / (wa[kk].abs() + 1e-3)).max())
            assert err <= 1e-5, (step, "activated", kk, err)
        # moments: torch keeps them per group
        st = opt.state[ref["delta"]]
        # (float32 rounding of m0 + (1 - beta1)(g - m0): absolute, at the scale of the array)
        for got, want_m in ((m["delta"], st["exp_avg"]), (v["delta"], st["exp_avg_sq"])):
            w = want_m.numpy()
            np.testing.assert_allclose(got.cpu().double().numpy(), w, rtol=1e-5, atol=1e-6 * np.abs(w).max())
    say(f"[adam n={n} K={k} D={deg}] three steps within 1e-5 of torch.optim.Adam (float64)")


@pytest.mark.parametrize("W,H,kind", [(64, 48, "noise"), (203, 131, "render"), (1920, 1080, "render-full")])
def test_ssim_loss_matches_oracle(R, W, H, kind):
    """Loss within 1e-5 relative; gradient per element within 1e-3 of the
    largest |dL/dx| (the SSIM map is float32 E[x^2] - mu^2 on the GPU)."""
    from oracle import losses
    from paper_2411_14974_amd import scenes
    rng = np.random.default_rng(W)
    if kind == "noise":
        x = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
        y = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
        x[:10, :10] = y[:10, :10]                     # identical patch
        x[20:30] = 0.5                                # flat band
    else:
        from paper_2411_14974_amd.binding import DeviceScene, make_params
        n = 20000 if kind == "render" else 200000
        scene, cam, target = scenes.config3(n=n, width=W, height=H)
        img, _ = R.forward(DeviceScene.from_scene(scene, "cuda:0"), cam, make_params())
        torch.cuda.synchronize()
        x = img.cpu().numpy()
        y = np.clip(x + rng.normal(0, 0.05, x.shape), 0, 1).astype(np.float32)
        y[: H // 4] = target[: H // 4]
    g, loss = R.ssim_loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    Lref, gref = losses.loss_and_grad(x.astype(np.float64), y.astype(np.float64))
    L = float(loss.cpu()[0])
    gg = g.cpu().numpy().astype(np.float64)
    err = float(np.abs(gg - gref).max() / np.abs(gref).max())
    say(f"[ssim {W}x{H} {kind}] loss {L:.7f} vs {Lref:.7f}; grad max err / max |g| {err:.1e}")
    assert abs(L - Lref) <= 1e-5 * abs(Lref)
    assert err <= 1e-3


@pytest.mark.parametrize("W,H", [(61, 37), (1920, 1080)])
def test_l1_loss_value_and_gradient(R, W, H):
    """mean |rgb - target| (added to the loss word) and sign(rgb - target) / n."""
    rng = np.random.default_rng(W)
    x = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
    y = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
    y[:5] = x[:5]  # ties: zero gradient
    loss = torch.full((1,), 0.5, device="cuda")
    g = R.l1_loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), loss=loss)
    torch.cuda.synchronize()
    want = float(np.abs(x.astype(np.float64) - y).mean())
    assert abs(float(loss.cpu()[0]) - 0.5 - want) <= 1e-5 * want
    np.testing.assert_array_equal(g.cpu().numpy(), np.sign(x - y).astype(np.float32) / np.float32(x.size))
