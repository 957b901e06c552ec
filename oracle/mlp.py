"""FP64 reference of the pair-policy network: a two-hidden-layer perceptron
with ReLU, masked mean-squared loss, its gradient by the chain rule, and one
Adam step (Kingma & Ba, 2015).  TEST INFRASTRUCTURE ONLY.

The network is not part of the paper: the paper's method chooses among its
approximations with a fixed operation-count rule (section 6, Figure 6) and
remarks that the cut-offs are rough; the library can replace that rule by a
learned cost predictor whose every choice is still certified by the paper's
error bounds.  This module is the plain definition the library's kernels are
checked against.

Parameter vector (float), in this order:
  W1[64][16], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]      (5508 values)
Forward, for an input x[16] already standardised:
  a1 = W1 x + b1,  h1 = max(a1, 0)
  a2 = W2 h1 + b2, h2 = max(a2, 0)
  y  = W3 h2 + b3
Loss over a batch, with targets t[n][4] and masks m[n][4] in {0, 1}:
  loss = sum_{n,k} m[n,k] (y[n,k] - t[n,k])^2 / max(1, sum m)
"""

import numpy as np

N_IN, N_HID, N_OUT = 16, 64, 4
SHAPES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta, X):
    """X[n][16] -> (y[n][4], cache)."""
    P = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ P["W3"].T + P["b3"]
    return y, (X, a1, h1, a2, h2)


def loss(theta, X, T, Mk):
    y, _ = forward(theta, X)
    Mk = np.asarray(Mk, dtype=np.float64)
    return float(np.sum(Mk * (y - T) ** 2) / max(1.0, float(Mk.sum())))


def gradient(theta, X, T, Mk):
    """d loss / d theta by the chain rule, packed like theta."""
    P = unpack(theta)
    y, (X, a1, h1, a2, h2) = forward(theta, X)
    Mk = np.asarray(Mk, dtype=np.float64)
    dy = 2.0 * Mk * (y - np.asarray(T, dtype=np.float64)) / max(1.0, float(Mk.sum()))
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    dh2 = (dy @ P["W3"]) * (a2 > 0.0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ P["W2"]) * (a1 > 0.0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(axis=0)
    return pack(g)


def adam_step(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; step counts from 1.  Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
