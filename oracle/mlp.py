"""FP64 reference of the child-ordering network (TEST INFRASTRUCTURE ONLY).

Used only by ``tests/`` (and nothing on the product path).  A plain numpy
statement of the network, its loss and its training step, written from their
textbook definitions:

  network   x (16) -> h1 = relu(W1 x + b1) (32) -> h2 = relu(W2 h1 + b2) (32)
            -> z = W3 h2 + b3 (4 logits, one per grandchild (u-half, v-half),
            index 2 * u_upper + v_upper)
  loss      mean over labelled samples of softmax cross-entropy,
            -z_y + log sum_k exp z_k; a sample with label 255 carries no label
  optimizer Adam (Kingma & Ba 2015) with bias correction

Parameters are one flat vector of 1732 values in the order W1 (32x16, row =
output unit), b1, W2 (32x32), b2, W3 (4x32), b3.

"bf16" mode states the reduced-precision arithmetic of the GPU network: the
input, the weights and each hidden activation (after the ReLU) are rounded to
bfloat16 (round to nearest, ties to even, from their fp32 value) and the sums
are exact; biases stay fp32.  Gradients then flow straight through the
roundings, i.e. they are those of the rounded network with respect to its
rounded weights, applied to the fp32 master weights.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 16, 32, 4
LAYOUT = (("W1", (32, 16)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (4, 32)), ("b3", (4,)))
N_PARAMS = 1732
NO_LABEL = 255


def unpack(theta: np.ndarray) -> dict:
    theta = np.asarray(theta, dtype=np.float64).reshape(-1)
    assert theta.size == N_PARAMS
    out, off = {}, 0
    for name, shape in LAYOUT:
        k = int(np.prod(shape))
        out[name] = theta[off:off + k].reshape(shape)
        off += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in LAYOUT])


def bf16_round(x) -> np.ndarray:
    """fp32 value of x rounded to bfloat16: keep the top 16 bits of the fp32
    pattern, rounding to nearest with ties to even (finite inputs)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def _weights(theta, bf16: bool) -> dict:
    p = unpack(theta)
    if bf16:
        for k in ("W1", "W2", "W3"):
            p[k] = bf16_round(p[k].astype(np.float32))
        for k in ("b1", "b2", "b3"):
            p[k] = p[k].astype(np.float32).astype(np.float64)
    return p


def forward(theta, X, bf16: bool = False):
    """Logits (n, 4) and the intermediate values of the pass."""
    p = _weights(theta, bf16)
    x = np.asarray(X, dtype=np.float64)
    if bf16:
        x = bf16_round(x.astype(np.float32))
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    if bf16:
        h1 = bf16_round(h1.astype(np.float32))
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    if bf16:
        h2 = bf16_round(h2.astype(np.float32))
    z = h2 @ p["W3"].T + p["b3"]
    return z, dict(p=p, x=x, a1=a1, h1=h1, a2=a2, h2=h2)


def softmax(z):
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def loss(theta, X, y, bf16: bool = False) -> float:
    z, _ = forward(theta, X, bf16)
    y = np.asarray(y).astype(np.int64)
    m = y != NO_LABEL
    if not m.any():
        return 0.0
    zm = z[m]
    lse = np.log(np.exp(zm - zm.max(axis=1, keepdims=True)).sum(axis=1)) + zm.max(axis=1)
    return float(np.mean(lse - zm[np.arange(zm.shape[0]), y[m]]))


def loss_and_grad(theta, X, y, bf16: bool = False):
    """Mean loss over the labelled samples and its gradient (backpropagation)."""
    z, c = forward(theta, X, bf16)
    p = c["p"]
    y = np.asarray(y).astype(np.int64)
    m = (y != NO_LABEL).astype(np.float64)
    cnt = max(1.0, m.sum())
    P = softmax(z)
    d3 = P.copy()
    d3[np.arange(len(y)), np.where(y == NO_LABEL, 0, y)] -= 1.0
    d3 *= m[:, None] / cnt
    g = {"W3": d3.T @ c["h2"], "b3": d3.sum(axis=0)}
    d2 = (d3 @ p["W3"]) * (c["a2"] > 0)
    g["W2"], g["b2"] = d2.T @ c["h1"], d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (c["a1"] > 0)
    g["W1"], g["b1"] = d1.T @ c["x"], d1.sum(axis=0)
    return loss(theta, X, y, bf16), pack(g)


def adam_step(theta, m, v, g, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based).  Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def predict_order(z):
    """(u-half, v-half) of the top-ranked grandchild (ties go to the lower index):
    the u-half is taken first, then that grandchild within it."""
    top = np.argmax(np.asarray(z), axis=1)
    return top >> 1, top & 1
