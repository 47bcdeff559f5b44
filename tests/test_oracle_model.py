"""Pins of the FP64 cost-model reference (central finite differences, the
closed form at zero weights, the first Adam step, descent on a full batch),
of the autotuner's selection rule, and of the brute-force plan model."""
import numpy as np
import pytest

from oracle import mlp, plan, tuner
from paper_2110_14340_amd import inputs


# ------------------------------------------------------------------ MLP
def _problem(F=12, B=32, seed=0):
    r = np.random.default_rng(seed)
    X = r.standard_normal((B, F))
    y = r.standard_normal(B)
    P = inputs.mlp_init(F, seed=seed + 100)
    P["b1"] = r.standard_normal(64) * 0.1
    P["b2"] = r.standard_normal(64) * 0.1
    P["b3"] = r.standard_normal(64) * 0.1
    P["b4"] = np.array([0.3])
    return P, X, y


def test_mlp_gradients_match_central_differences():
    P, X, y = _problem()
    L, g = mlp.gradients(P, X, y)
    assert abs(L - mlp.loss(P, X, y)) <= 1e-15 * L
    h = 1e-6
    r = np.random.default_rng(1)
    for name in mlp.PARAM_NAMES:
        flat = P[name].reshape(-1)
        idx = r.choice(flat.size, size=min(6, flat.size), replace=False)
        for k in idx:
            Pp = {n: v.copy() for n, v in P.items()}
            Pm = {n: v.copy() for n, v in P.items()}
            Pp[name].reshape(-1)[k] += h
            Pm[name].reshape(-1)[k] -= h
            fd = (mlp.loss(Pp, X, y) - mlp.loss(Pm, X, y)) / (2 * h)
            an = g[name].reshape(-1)[k]
            assert abs(fd - an) <= 1e-6 * max(abs(fd), abs(an), 1e-3), (name, k, fd, an)


def test_mlp_zero_weights_closed_form():
    F = 7
    P = {k: np.zeros(s) for k, s in mlp.shapes(F).items()}
    P["b4"] = np.array([0.25])
    X = np.random.default_rng(2).standard_normal((16, F))
    y = np.random.default_rng(3).standard_normal(16)
    L, g = mlp.gradients(P, X, y)
    assert np.isclose(L, np.mean((0.25 - y) ** 2), rtol=1e-15)
    assert np.isclose(g["b4"][0], 2 * np.mean(0.25 - y), rtol=1e-14)
    for k in mlp.PARAM_NAMES:
        if k != "b4":
            assert np.all(g[k] == 0.0), k


def test_relu_derivative_at_zero_is_zero():
    # a pre-activation exactly 0 must pass no gradient
    F = 2
    P = {k: np.zeros(s) for k, s in mlp.shapes(F).items()}
    P["w4"] = np.ones(64)
    P["W3"] = np.zeros((64, 64))
    P["b3"] = np.zeros(64)   # z3 == 0 exactly
    X = np.ones((4, F))
    _, g = mlp.gradients(P, X, np.zeros(4))
    assert np.all(g["W3"] == 0) and np.all(g["b3"] == 0)


def test_adam_first_step_is_lr_times_sign():
    P = {"w": np.array([0.5, -1.0, 2.0])}
    g = {"w": np.array([3.0, -0.02, 1e-3])}
    opt = mlp.Adam(P)
    out = opt.step(P, g)
    # m_hat = g, v_hat = g^2 after one step: p - lr * g / (|g| + eps)
    expect = P["w"] - 1e-3 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(out["w"], expect, rtol=0, atol=1e-15)


def test_full_batch_descent_lowers_loss():
    P, X, y = _problem(seed=4)
    opt = mlp.Adam(P, lr=1e-3)
    L0 = mlp.loss(P, X, y)
    for _ in range(200):
        _, g = mlp.gradients(P, X, y)
        P = opt.step(P, g)
    assert mlp.loss(P, X, y) < 0.5 * L0


def test_standardise_constant_feature():
    X = np.array([[1.0, 5.0], [3.0, 5.0]])
    mu, sd = mlp.standardise_stats(X)
    assert np.array_equal(mu, [2.0, 5.0]) and np.array_equal(sd, [1.0, 1.0])


# ------------------------------------------------------------------ tuner
def test_tuner_select_median_and_ties():
    samples = [[5, 1, 9], [2, 3, 100], [3, 2, 2.5], [2.5, 2.5, 9]]
    # medians: 5, 3, 2.5, 2.5 -> tie between 2 and 3 goes to 2
    assert tuner.select(samples) == 2
    assert tuner.median([4, 1, 3, 2]) == 2.5
    assert tuner.regret(1.05, 1.0) == pytest.approx(0.05)


# ------------------------------------------------------------------ plan
def test_blocks_cover_and_are_disjoint():
    for E in range(1, 40):
        for K in range(1, E + 1):
            rows = []
            for p in range(K):
                rows.extend(range(*plan.block(E, K, p)))
            assert rows == list(range(E))


def test_jacobi_8192_k8_plan():
    E, K = 8192, 8
    A = {"in": plan.ArrayState(E, K, 1, 1), "out": plan.ArrayState(E, K, 1, 1)}
    args = [("in", "r", -1, 1, False), ("out", "w", 0, 0, False)]
    ps = plan.plan_loop(A, 1, E - 1, args)
    assert min(ps[0]["I"]) == 1 and max(ps[0]["I"]) == 1023
    assert min(ps[7]["I"]) == 7168 and max(ps[7]["I"]) == 8190
    assert ps[3]["reads"]["in"] == set(range(3 * 1024 - 1, 4 * 1024 + 1))
    assert all(p["copies"] == [] for p in ps)   # fresh after enter
    # the next sweep reads "out": every interior boundary needs its two rows
    ps2 = plan.plan_loop(A, 1, E - 1, [("out", "r", -1, 1, False), ("in", "w", 0, 0, False)])
    copies = [c for p in ps2 for c in p["copies"]]
    assert len(copies) == 14
    assert ("out", 0, 1023, 1024) in ps2[1]["copies"] and ("out", 2, 2048, 2049) in ps2[1]["copies"]


def test_plan_rejects_overlapping_writes_and_out_of_slab():
    A = {"a": plan.ArrayState(16, 4, 0, 0)}
    with pytest.raises(ValueError):
        plan.plan_loop(A, 1, 15, [("a", "r", -1, 1, False)])   # no halo declared
    B = {"a": plan.ArrayState(16, 4, 1, 1), "b": plan.ArrayState(16, 4, 1, 1)}
    with pytest.raises(ValueError):
        plan.plan_loop(B, 0, 16, [("a", "r", 0, 0, False), ("b", "w", 0, 1, False)])
