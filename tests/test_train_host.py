"""Host-side training helpers: the exponential position learning rate."""
import math

from paper_2411_14974_amd import binding


def test_expon_lr_endpoints_and_geometric_midpoint():
    assert math.isclose(binding.expon_lr(0), 5e-4, rel_tol=1e-12)
    assert math.isclose(binding.expon_lr(30_000), 5e-6, rel_tol=1e-12)
    assert math.isclose(binding.expon_lr(90_000), 5e-6, rel_tol=1e-12)  # constant after the decay
    # log-linear: the midpoint is the geometric mean of the endpoints
    assert math.isclose(binding.expon_lr(15_000), math.sqrt(5e-4 * 5e-6), rel_tol=1e-12)
    lrs = [binding.expon_lr(s) for s in range(0, 30_001, 1000)]
    assert all(a > b for a, b in zip(lrs, lrs[1:]))


def test_adam_params_struct():
    p = binding.make_adam_params(7)
    assert p.step == 7 and math.isclose(p.lr_points, binding.expon_lr(7), rel_tol=1e-6)
    assert math.isclose(p.lr_delta, 0.005, rel_tol=1e-6) and math.isclose(p.lr_sigma, 0.0045, rel_tol=1e-6)
