"""FP64 reference of the learned pre-screen (oracle; test infrastructure only).

A 4-layer perceptron over a candidate's action bitmask and an injection
summary:

    z1 = sum_{i in bits} W1b[i] + x_dense W1d + b1,   h1 = relu(z1)
    z2 = h1 W2 + b2,                                   h2 = relu(z2)
    z3 = h2 W3 + b3,                                   h3 = relu(z3)
    y  = h3 W4 + b4                                    (two outputs)

Loss L = 1/(2B) sum_b sum_k (y_bk - t_bk)^2, trained with Adam (bias-corrected
first and second moments, as published by Kingma and Ba).  The paper has no
learned component; this network and its targets (maximum loading and
log-overload) follow the surrogate workload description.  Written straight
from the chain rule, in float64, for small batches.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

PARAM_NAMES = ["W1b", "W1d", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]


def relu(x):
    return np.maximum(x, 0.0)


def forward(p: Dict[str, np.ndarray], bits: List[np.ndarray], dense: np.ndarray,
            act_round=None):
    """Returns y [B, 2] and the cache of pre-activations/activations.

    act_round, if given, is applied to every hidden activation: a network
    specified with activations stored in a narrower type (BF16) is then the
    same function here, and its ReLU decisions are taken on the same values.
    The backward pass treats the rounding as the identity."""
    rnd = (lambda v: v) if act_round is None else act_round
    B = len(bits)
    z1 = dense @ p["W1d"] + p["b1"][None, :]
    for b in range(B):
        for i in bits[b]:
            z1[b] += p["W1b"][int(i)]
    h1 = rnd(relu(z1))
    z2 = h1 @ p["W2"] + p["b2"][None, :]
    h2 = rnd(relu(z2))
    z3 = h2 @ p["W3"] + p["b3"][None, :]
    h3 = rnd(relu(z3))
    y = h3 @ p["W4"] + p["b4"][None, :]
    return y, dict(z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3)


def loss(y: np.ndarray, t: np.ndarray) -> float:
    return float(0.5 * ((y - t) ** 2).sum() / y.shape[0])


def backward(p, bits, dense, cache, y, t) -> Dict[str, np.ndarray]:
    """Gradients of the loss with respect to every parameter."""
    B = y.shape[0]
    g = {}
    dy = (y - t) / B
    g["W4"] = cache["h3"].T @ dy
    g["b4"] = dy.sum(axis=0)
    dz3 = (dy @ p["W4"].T) * (cache["z3"] > 0)
    g["W3"] = cache["h2"].T @ dz3
    g["b3"] = dz3.sum(axis=0)
    dz2 = (dz3 @ p["W3"].T) * (cache["z2"] > 0)
    g["W2"] = cache["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * (cache["z1"] > 0)
    g["W1d"] = dense.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    gw = np.zeros_like(p["W1b"])
    for b in range(B):
        for i in bits[b]:
            gw[int(i)] += dz1[b]
    g["W1b"] = gw
    return g


@dataclass
class AdamState:
    m: Dict[str, np.ndarray]
    v: Dict[str, np.ndarray]
    step: int = 0


def adam_init(p) -> AdamState:
    return AdamState(m={k: np.zeros_like(v) for k, v in p.items()},
                     v={k: np.zeros_like(v) for k, v in p.items()})


def adam_step(p, g, st: AdamState, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (in place on p and st)."""
    st.step += 1
    c1 = 1.0 - beta1 ** st.step
    c2 = 1.0 - beta2 ** st.step
    for k in p:
        st.m[k] = beta1 * st.m[k] + (1.0 - beta1) * g[k]
        st.v[k] = beta2 * st.v[k] + (1.0 - beta2) * g[k] * g[k]
        mh = st.m[k] / c1
        vh = st.v[k] / c2
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
