"""FP64 reference of the learned cost model (test infrastructure only).

The network maps a standardised feature vector x (F values) of one loop nest
and one launch configuration to a predicted log run time:

    h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3)
    yhat = w4 . h3 + b4

with three hidden layers of width 64.  The loss over a batch is the mean of
(yhat - y)^2 with y = log(time).  Gradients follow the chain rule with the
convention relu'(0) = 0.  The optimiser is Adam with bias correction.

The paper has no learned model; auto-tuning is named as future work in its
conclusion.  This module is the plain definition the GPU kernels are
checked against (FP32 on the GPU, FP64 here).
"""
import numpy as np

HIDDEN = 64
PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4")


def shapes(F, H=HIDDEN):
    return {"W1": (H, F), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H, H), "b3": (H,),
            "w4": (H,), "b4": (1,)}


def forward(params, X):
    """Returns (yhat [B], cache)."""
    P = {k: np.asarray(v, dtype=np.float64) for k, v in params.items()}
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.where(z1 > 0, z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.where(z2 > 0, z2, 0.0)
    z3 = h2 @ P["W3"].T + P["b3"]
    h3 = np.where(z3 > 0, z3, 0.0)
    yhat = h3 @ P["w4"] + P["b4"][0]
    return yhat, (X, z1, h1, z2, h2, z3, h3)


def loss(params, X, y):
    yhat, _ = forward(params, X)
    d = yhat - np.asarray(y, dtype=np.float64)
    return float(np.mean(d * d))


def gradients(params, X, y):
    """Returns (loss, dict of gradients with the parameters' shapes)."""
    P = {k: np.asarray(v, dtype=np.float64) for k, v in params.items()}
    yhat, (X, z1, h1, z2, h2, z3, h3) = forward(P, X)
    B = X.shape[0]
    d = yhat - np.asarray(y, dtype=np.float64)
    L = float(np.mean(d * d))
    gy = 2.0 * d / B                       # dL/dyhat
    g = {}
    g["w4"] = h3.T @ gy
    g["b4"] = np.array([gy.sum()])
    gz3 = np.outer(gy, P["w4"]) * (z3 > 0)
    g["W3"] = gz3.T @ h2
    g["b3"] = gz3.sum(axis=0)
    gz2 = (gz3 @ P["W3"]) * (z2 > 0)
    g["W2"] = gz2.T @ h1
    g["b2"] = gz2.sum(axis=0)
    gz1 = (gz2 @ P["W2"]) * (z1 > 0)
    g["W1"] = gz1.T @ X
    g["b1"] = gz1.sum(axis=0)
    return L, g


class Adam:
    """Adam with bias correction: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(np.asarray(v, dtype=np.float64)) for k, v in params.items()}
        self.v = {k: np.zeros_like(np.asarray(v, dtype=np.float64)) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = {}
        for k in params:
            p = np.asarray(params[k], dtype=np.float64)
            gk = grads[k]
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * gk
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * gk * gk
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            out[k] = p - self.lr * mh / (np.sqrt(vh) + self.eps)
        return out


def standardise_stats(X):
    """Mean and standard deviation per feature over the training rows (a
    zero deviation is replaced by 1 so a constant feature maps to 0)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return mu, sd
