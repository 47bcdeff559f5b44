"""GPU parity of the learned cost model's hand-written FP32 kernels against
the FP64 oracle (forward output and every gradient tensor within 1e-4
relative in L2 for the same weights and batch), the zero-weight closed form,
the first Adam step, and descent of the training loop."""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2110_14340_amd import inputs, jacc
from gpu_util import context, say

pytestmark = pytest.mark.gpu


def _problem(F, B, seed):
    r = np.random.default_rng(seed)
    X = r.standard_normal((B, F)).astype(np.float32)
    y = r.standard_normal(B).astype(np.float32)
    P = inputs.mlp_init(F, seed=seed + 1)
    for k in ("b1", "b2", "b3"):
        P[k] = r.standard_normal(64) * 0.1
    P["b4"] = np.array([0.2])
    P32 = {k: np.asarray(v, dtype=np.float32) for k, v in P.items()}
    return X, y, P32


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("F,B", [(12, 64), (12, 257), (5, 3), (16, 128)])
def test_forward_and_gradients_match_fp64_oracle(F, B):
    say(f"mlp gradients F={F} B={B}")
    X, y, P = _problem(F, B, seed=F * 100 + B)
    ref_P = {k: v.astype(np.float64) for k, v in P.items()}
    with context(1) as c:
        m = jacc.Model(c, F)
        m.set_params(P)
        yhat = m.predict(X)
        loss, g = m.gradients(X, y)
        got_P = m.get_params()
        m.close()
    for k in P:
        assert np.array_equal(got_P[k], P[k])
    ref_yhat, _ = omlp.forward(ref_P, X.astype(np.float64))
    assert _rel(yhat, ref_yhat) <= 1e-4
    ref_loss, ref_g = omlp.gradients(ref_P, X.astype(np.float64), y.astype(np.float64))
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    for k in omlp.PARAM_NAMES:
        assert _rel(g[k], ref_g[k]) <= 1e-4, k


def test_scaler_is_applied_inside_forward():
    say("mlp scaler")
    F, B = 12, 50
    X, y, P = _problem(F, B, seed=3)
    X = X * 7.0 + 3.0
    mu = X.mean(axis=0).astype(np.float32)
    sd = X.std(axis=0).astype(np.float32)
    with context(1) as c:
        m = jacc.Model(c, F)
        m.set_params(P)
        m.set_scaler(mu, sd)
        yhat = m.predict(X)
        m.close()
    Xs = (X.astype(np.float64) - mu) / sd
    ref, _ = omlp.forward({k: v.astype(np.float64) for k, v in P.items()}, Xs)
    assert _rel(yhat, ref) <= 1e-4


def test_zero_weights_closed_form():
    say("mlp zero weights")
    F, B = 7, 33
    r = np.random.default_rng(4)
    X = r.standard_normal((B, F)).astype(np.float32)
    y = r.standard_normal(B).astype(np.float32)
    with context(1) as c:
        m = jacc.Model(c, F)
        P = {k: np.zeros(s, dtype=np.float32) for k, s in m.shapes().items()}
        P["b4"] = np.array([0.25], dtype=np.float32)
        m.set_params(P)
        loss, g = m.gradients(X, y)
        m.close()
    assert abs(g["b4"][0] - 2.0 * np.mean(0.25 - y.astype(np.float64))) <= 1e-5
    for k in omlp.PARAM_NAMES:
        if k != "b4":
            assert np.all(g[k] == 0.0), k
    assert abs(loss - np.mean((0.25 - y.astype(np.float64)) ** 2)) <= 1e-5


def test_adam_step_matches_oracle():
    say("mlp adam step")
    F, B = 12, 40
    X, y, P = _problem(F, B, seed=5)
    with context(1) as c:
        m = jacc.Model(c, F)
        m.set_params(P)
        _, g = m.gradients(X, y)
        m.adam_step(1e-3)
        got = m.get_params()
        m.close()
    opt = omlp.Adam({k: v.astype(np.float64) for k, v in P.items()})
    ref = opt.step({k: v.astype(np.float64) for k, v in P.items()}, {k: np.asarray(v, np.float64) for k, v in g.items()})
    for k in P:
        assert np.allclose(got[k], ref[k], rtol=0, atol=2e-6), k


def test_training_lowers_loss_and_generalises():
    say("mlp training")
    F = 12
    r = np.random.default_rng(6)
    X = r.standard_normal((3000, F))
    w = r.standard_normal(F)
    y = np.log1p(np.exp(X @ w * 0.5)) + 0.1 * np.sin(3 * X[:, 0])
    with context(1) as c:
        m = jacc.Model(c, F)
        m.set_params(inputs.mlp_init(F, seed=7))
        m.set_scaler(X.mean(axis=0), X.std(axis=0))
        losses = m.train(X[:2500], y[:2500], epochs=60, batch=256, lr=1e-3, seed=1)
        pred = m.predict(X[2500:])
        m.close()
    assert losses[-1] < 0.2 * losses[0]
    assert np.mean((pred - y[2500:]) ** 2) < 0.2 * np.var(y[2500:])
