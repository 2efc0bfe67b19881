"""Pins for the change-predictor network oracle (oracle/mlp.py): bf16 rounding
against hand-worked cases of the format, gradients against central finite
differences, Adam's first step against its closed form.  No GPU."""
import numpy as np
import pytest

from oracle import mlp


def _bits(x):
    return np.asarray(x, dtype=np.float32).view(np.uint32)


def test_bf16_round_ties_and_fixed_points():
    one = 1.0
    cases = {
        one: one,
        one + 2.0 ** -8: one,                    # halfway, even neighbour is 1.0
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,    # halfway, even neighbour above
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,  # just above halfway
        -(one + 2.0 ** -8): -one,
        one + 2.0 ** -7: one + 2.0 ** -7,        # representable
        3.0e38: np.inf if np.float32(3.0e38) > np.float32(3.3895e38) else None,
    }
    for x, want in cases.items():
        if want is None:
            continue
        got = mlp.bf16_round(np.float32(x)).item()
        assert got == np.float32(want), (x, got, want)
    # the largest finite float rounds up to infinity (RNE carries into the exponent)
    assert np.isinf(mlp.bf16_round(np.float32(np.finfo(np.float32).max)))
    assert np.isnan(mlp.bf16_round(np.float32(np.nan)))


def test_bf16_round_properties():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200000) * 10.0 ** rng.uniform(-10, 10, 200000)).astype(np.float32)
    r = mlp.bf16_round(x)
    assert np.all(_bits(r) & 0xFFFF == 0)                 # a bfloat16 value
    assert np.array_equal(mlp.bf16_round(r), r)            # idempotent
    # within half a unit in the last place of bfloat16 (8 significant bits)
    ulp = np.ldexp(1.0, np.frexp(np.abs(x).astype(np.float64))[1] - 8)
    assert np.all(np.abs(r.astype(np.float64) - x) <= ulp / 2 + 1e-300)


def test_bce_special_values():
    assert mlp.bce_loss([0.0], [1.0]) == pytest.approx(np.log(2.0))
    assert mlp.bce_loss([0.0], [0.0]) == pytest.approx(np.log(2.0))
    assert mlp.bce_loss([0.0], [1.0], pos_weight=3.0) == pytest.approx(3.0 * np.log(2.0))
    z = np.array([-3.0, 0.5, 4.0])
    y = np.array([0.0, 1.0, 1.0])
    s = 1.0 / (1.0 + np.exp(-z))
    want = np.mean(-(2.0 * y * np.log(s) + (1 - y) * np.log(1 - s)))
    assert mlp.bce_loss(z, y, pos_weight=2.0) == pytest.approx(want, rel=1e-12)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(3)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, size=p[k].shape).astype(np.float32)
    p = {k: v.astype(np.float64) for k, v in p.items()}
    X = rng.normal(size=(16, mlp.N_IN))
    y = (rng.random(16) < 0.3).astype(np.float64)
    g = mlp.backward(p, X, y, pos_weight=2.5, exact=True)
    h = 1e-6
    for k in mlp.PARAM_ORDER:
        flat = p[k].ravel()
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = mlp.bce_loss(mlp.forward(p, X, exact=True)[0], y, 2.5)
            flat[i] = old - h
            lm = mlp.bce_loss(mlp.forward(p, X, exact=True)[0], y, 2.5)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert g[k].ravel()[i] == pytest.approx(fd, rel=1e-5, abs=1e-8), (k, i)


def test_adam_first_step_closed_form():
    # with m0 = v0 = 0 and t = 1 the bias-corrected moments are g and g^2, so
    # the step is lr * g / (|g| + eps)
    p = {k: np.full(s, 0.5, dtype=np.float32) for k, s in mlp.PARAM_SHAPES.items()}
    rng = np.random.default_rng(2)
    g = {k: rng.normal(size=s) for k, s in mlp.PARAM_SHAPES.items()}
    m = {k: np.zeros(s, np.float32) for k, s in mlp.PARAM_SHAPES.items()}
    v = {k: np.zeros(s, np.float32) for k, s in mlp.PARAM_SHAPES.items()}
    p0 = {k: x.copy() for k, x in p.items()}
    mlp.adam_step(p, g, m, v, t=1, lr=1e-2)
    for k in mlp.PARAM_ORDER:
        gk = np.asarray(g[k], dtype=np.float32).astype(np.float64)
        want = p0[k].astype(np.float64) - 1e-2 * gk / (np.abs(gk) + 1e-8)
        assert np.allclose(p[k], want, rtol=0, atol=2e-7), k


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(512, mlp.N_IN)).astype(np.float32)
    y = ((X[:, 0] + 0.5 * X[:, 3]) > 0.3).astype(np.float64)
    p = mlp.init_params(5)
    m = {k: np.zeros_like(x) for k, x in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    l0 = mlp.bce_loss(mlp.forward(p, X)[0], y)
    for t in range(1, 201):
        mlp.adam_step(p, mlp.backward(p, X, y), m, v, t, lr=3e-3)
    l1 = mlp.bce_loss(mlp.forward(p, X)[0], y)
    assert l1 < 0.5 * l0


def test_parameter_count():
    assert mlp.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5057
    p = mlp.init_params(0)
    assert all(np.array_equal(a, b) for a, b in
               zip(mlp.unflatten(mlp.flatten(p)).values(), p.values()))
