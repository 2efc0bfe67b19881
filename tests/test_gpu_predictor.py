"""GPU parity of the change-predictor network (liblpa.so, through the C ABI)
against the fp64 oracle in oracle/mlp.py.

Tolerances follow from the arithmetic.  The training kernel computes in fp32
on the same bf16-rounded weights and inputs as the oracle, so logits and
gradients agree to fp32 summation error (relative 1e-4 of the largest term,
with slack for atomics' order).  Inference runs on MFMA with bf16 hidden
first-layer activations; a fp32 accumulation landing on the other side of a
bf16 rounding boundary moves one hidden value by one bf16 ulp (2^-8
relative), so logits are compared against the oracle with bf16 first-layer
rounding at 2e-2 absolute + 1e-2 relative, and on average far tighter.  Adam is elementwise fp32 against
fp64, so one fp32 ulp of the parameter.
"""
import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2411_11468_amd import lpa  # noqa: E402


def _samples(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((n, mlp.N_IN)) * scale).astype(np.float32)
    y = (rng.random(n) < 0.3).astype(np.float32)
    return X, y


def _params(seed):
    p = mlp.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    for k in ("b1", "b2", "b3"):
        p[k] = (rng.standard_normal(p[k].shape) * 0.1).astype(np.float32)
    return p


@pytest.mark.parametrize("n", [1, 63, 64, 1000])
def test_gradient_matches_oracle(n):
    p = _params(3)
    X, y = _samples(n, 5)
    pr = lpa.Predictor(params=mlp.flatten(p))
    g, loss = pr.gradient(X, y, pos_weight=2.5)
    z, _ = mlp.forward(p, X)
    want_loss = mlp.bce_loss(z, y, 2.5)
    assert loss == pytest.approx(want_loss, rel=1e-5, abs=1e-6)
    want = mlp.flatten({k: np.asarray(v) for k, v in mlp.backward(p, X, y, 2.5).items()})
    scale = np.abs(want).max()
    np.testing.assert_allclose(g, want, rtol=1e-4, atol=1e-5 * scale)
    pr.close()


def test_gradient_device_inputs_and_empty():
    p = _params(7)
    X, y = _samples(300, 8)
    pr = lpa.Predictor(params=mlp.flatten(p))
    g_host, l_host = pr.gradient(X, y)
    g_dev, l_dev = pr.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda())
    np.testing.assert_allclose(g_dev, g_host, rtol=1e-5, atol=1e-7)
    assert l_dev == pytest.approx(l_host, rel=1e-6)
    g0, l0 = pr.gradient(X[:0], y[:0])
    assert not g0.any() and l0 == 0.0
    pr.close()


def test_adam_matches_oracle():
    p = _params(11)
    X, y = _samples(500, 12)
    pr = lpa.Predictor(params=mlp.flatten(p))
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    for t in range(1, 4):
        g = mlp.backward(p, X, y, 1.0)
        gflat = mlp.flatten({k: np.asarray(a, dtype=np.float32) for k, a in g.items()})
        pr.adam(gflat, lr=1e-3)
        mlp.adam_step(p, {k: np.asarray(a, dtype=np.float32) for k, a in g.items()}, m, v, t,
                      lr=1e-3)
        got = pr.params()
        want = mlp.flatten(p)
        np.testing.assert_allclose(got, want, rtol=2e-7, atol=2e-9)
        p = mlp.unflatten(got)   # continue from the GPU's own parameters
    pr.close()


def test_set_get_roundtrip_and_create_seeded():
    a = lpa.Predictor(seed=42)
    b = lpa.Predictor(seed=42)
    pa, pb = a.params(), b.params()
    np.testing.assert_array_equal(pa, pb)
    assert pa.shape == (mlp.N_PARAMS,)
    # weights He-uniform in +-sqrt(6/fan_in), biases zero
    d = mlp.unflatten(pa)
    assert np.abs(d["W1"]).max() <= np.sqrt(6 / 12) and np.abs(d["W2"]).max() <= np.sqrt(6 / 64)
    assert not d["b1"].any() and not d["b2"].any() and not d["b3"].any()
    q = mlp.flatten(_params(1))
    a.set_params(q)
    np.testing.assert_array_equal(a.params(), q)
    a.close()
    b.close()


@pytest.mark.parametrize("n", [1, 15, 16, 17, 4099])
def test_predict_matches_oracle(n):
    p = _params(21)
    X, _ = _samples(n, 22, scale=2.0)
    pr = lpa.Predictor(params=mlp.flatten(p))
    prob = pr.predict(X)
    z, _ = mlp.forward(p, X, bf16_h1=True)
    zg = np.log(prob.astype(np.float64)) - np.log1p(-prob.astype(np.float64))
    ok = np.abs(prob - mlp.sigmoid(z)) < 1e-6     # saturated probabilities
    err = np.abs(zg - z)
    assert np.all(ok | (err <= 2e-2 + 1e-2 * np.abs(z)))
    # a bf16 rounding flip of a first-layer activation is rare: nearly every
    # logit agrees to fp32 summation error
    if (~ok).any():
        assert np.mean(err[~ok] > 1e-4) <= max(0.05, 1.0 / n)
    # device in, device out
    pd = pr.predict(torch.from_numpy(X).cuda())
    np.testing.assert_array_equal(pd.cpu().numpy(), prob)
    pr.close()


def test_full_batch_training_matches_oracle():
    """With one batch per epoch the sample order is irrelevant, so the GPU's
    training loop must follow the oracle's gradient + Adam steps."""
    p = _params(31)
    X, y = _samples(777, 32)
    pr = lpa.Predictor(params=mlp.flatten(p))
    epochs, lr = 4, 1e-3
    loss = pr.train(X, y, epochs=epochs, batch=len(y), lr=lr, pos_weight=1.5, seed=3)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    for t in range(1, epochs + 1):
        z, _ = mlp.forward(p, X)
        want_loss = mlp.bce_loss(z, y, 1.5)
        g = mlp.backward(p, X, y, 1.5)
        mlp.adam_step(p, {k: np.asarray(a, dtype=np.float32) for k, a in g.items()}, m, v, t,
                      lr=lr)
    assert loss == pytest.approx(want_loss, rel=1e-4)
    got, want = pr.params(), mlp.flatten(p)
    # Adam normalises each step to about lr, so a gradient within fp32 error
    # of zero may take either sign: allow that on a few parameters
    close = np.abs(got - want) <= 1e-6 + 1e-5 * np.abs(want)
    assert close.mean() > 0.99
    assert np.abs(got - want).max() <= 2 * lr * epochs + 1e-6
    pr.close()


def test_training_learns_a_separable_rule():
    rng = np.random.default_rng(41)
    X = rng.standard_normal((20000, mlp.N_IN)).astype(np.float32)
    y = ((X[:, 0] + 0.5 * X[:, 1] - X[:, 2]) > 0.3).astype(np.float32)
    pr = lpa.Predictor(seed=5)
    first = pr.train(X, y, epochs=1, batch=256, lr=3e-3, seed=1)
    last = pr.train(X, y, epochs=5, batch=256, lr=3e-3, seed=2)
    assert last < 0.5 * first
    Xt = rng.standard_normal((5000, mlp.N_IN)).astype(np.float32)
    yt = ((Xt[:, 0] + 0.5 * Xt[:, 1] - Xt[:, 2]) > 0.3)
    acc = np.mean((pr.predict(Xt) > 0.5) == yt)
    assert acc > 0.95
    pr.close()


def test_predictor_invalid_arguments():
    pr = lpa.Predictor(seed=1)
    with pytest.raises(ValueError):
        pr.set_params(np.zeros(10, dtype=np.float32))
    X, y = _samples(10, 1)
    with pytest.raises(lpa.LpaError):
        pr.train(X, y, epochs=1, batch=0)
    with pytest.raises(lpa.LpaError):
        pr.train(X, y, epochs=1, batch=4, lr=0.0)
    pr.close()


def test_save_load_checkpoint_resumes_training():
    # lpa_predictor_save / lpa_predictor_load: shape header, parameters and
    # Adam state.  A loaded predictor holds exactly the saved state (its own
    # blob is the same bytes, its predictions the same values); trained on,
    # it follows the saved one up to the order of the gradient kernel's
    # float atomic sums, far closer than a predictor given only the
    # parameters, whose Adam state starts at zero
    X, y = _samples(4000, 7)
    a = lpa.Predictor(seed=3)
    a.train(X, y, epochs=1, batch=256, lr=2e-3, seed=1)
    blob = a.save_blob()
    assert len(blob) == 32 + 3 * 4 * lpa.PREDICTOR_PARAMS
    assert blob[:8] == b"LPAPRED1"
    b = lpa.Predictor(seed=99)
    b.load_blob(blob)
    assert b.save_blob() == blob
    np.testing.assert_array_equal(a.params(), b.params())
    pa, pb = a.predict(X), b.predict(X)
    np.testing.assert_array_equal(np.asarray(pa.cpu() if hasattr(pa, "cpu") else pa),
                                  np.asarray(pb.cpu() if hasattr(pb, "cpu") else pb))
    c = lpa.Predictor(seed=99)
    c.set_params(np.frombuffer(blob[32:32 + 4 * lpa.PREDICTOR_PARAMS], dtype=np.float32))
    la = a.train(X, y, epochs=2, batch=256, lr=2e-3, seed=5)
    lb = b.train(X, y, epochs=2, batch=256, lr=2e-3, seed=5)
    c.train(X, y, epochs=2, batch=256, lr=2e-3, seed=5)
    assert abs(la - lb) <= 1e-5 * abs(la)
    # quantiles, not maxima: a parameter whose gradient is pure cancellation
    # may take an Adam step of either sign in either run
    d_ab = float(np.quantile(np.abs(a.params() - b.params()), 0.99))
    d_ac = float(np.quantile(np.abs(a.params() - c.params()), 0.5))
    print(f"99th percentile |a-b| {d_ab:.3g}, median |a-c| {d_ac:.3g}")
    assert d_ac >= 1e-4
    assert d_ab <= 0.02 * d_ac
    # corrupted or foreign blobs are refused and leave the predictor as it was
    before = b.params()
    bad = [b"XXXXXXXX" + blob[8:], blob[:100], blob[:8] + b"\x02" + blob[9:],
           blob[:12] + b"\x0d" + blob[13:]]
    nan = bytearray(blob)
    nan[32:36] = np.array([np.nan], np.float32).tobytes()
    bad.append(bytes(nan))
    for x in bad:
        with pytest.raises(lpa.LpaError):
            b.load_blob(x)
    np.testing.assert_array_equal(b.params(), before)
    for p in (a, b, c):
        p.close()
