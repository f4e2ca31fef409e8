"""Reference message-passing network for learned smooth-error proposals.

Test infrastructure only (like the rest of ``oracle``): plain numpy, written
for reading, not speed.  It defines the learned extension's network; the
library's HIP kernels must reproduce it.

The method builds its path cover from keys |e_i - e_j| of a smooth error e
(Alg. 4, Step 2; Sec. 3.2); the extension replaces most of the relaxation
sweeps that produce e by a network that maps a briefly relaxed vector to a
smoother one.  Keys depend only on the level sets of e, so the network
predicts a node vector and the edge order follows from it.

Graph: symmetric CSR (rp, ci, w) of the weighted graph, d_i = sum_j w_ij,
normalised adjacency Ahat = D^{-1} W (row i: w_ij / d_i).

Features (n x 4, float32): with u = normalise(e2) (mean removed, unit RMS)
and l_i = log d_i - mean(log d):  F = [u, Ahat u, l, Ahat l].

Network (hidden 64, three message-passing layers):
    h0 = relu(F W0 + b0)                      W0: 4 x 64      (float32)
    for k = 1..3:
        z_k = [h_{k-1} | Ahat h_{k-1}]        n x 128
        h_k = relu(bf(z_k) bf(W_k) + b_k)     W_k: 128 x 64   (bf16 x bf16 -> float32)
    y = h3 wo + bo + u                        wo: 64          (float32)
Loss against a target t (normalised like u): L = 0.5 * mean((y - t)^2).

bf(.) rounds float32 to bfloat16 (round to nearest, ties to even) when
``bf16`` is on; backward products use bf16 operands the same way
(dZ = bf(dP) bf(W)^T, dW = bf(Z)^T bf(dP)), float32 accumulation.
Parameter vector order: W0, b0, (W_k, b_k) for k = 1..3, wo, bo.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

HIDDEN = 64
NFEAT = 4
LAYERS = 3
SHAPES = [(NFEAT, HIDDEN), (HIDDEN,)] + [(2 * HIDDEN, HIDDEN), (HIDDEN,)] * LAYERS + [(HIDDEN,), (1,)]
NPARAMS = int(sum(np.prod(s) for s in SHAPES))


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def unpack(theta: np.ndarray):
    out, k = [], 0
    for s in SHAPES:
        m = int(np.prod(s))
        out.append(np.asarray(theta[k:k + m]).reshape(s))
        k += m
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases (float32 values)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, s))
        elif s == (HIDDEN,) and len(parts) == 2 * LAYERS + 2:  # wo
            parts.append(rng.uniform(-0.1, 0.1, s))
        else:
            parts.append(np.zeros(s))
    return pack(parts).astype(np.float32)


def normalise(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    c = v - v.mean()
    r = np.sqrt(np.mean(c * c))
    return c / r if r > 0 else c


def graph_ops(g):
    n, rp, ci, w = g
    W = sp.csr_matrix((np.asarray(w, np.float64), np.asarray(ci), np.asarray(rp)), shape=(n, n))
    d = np.asarray(W.sum(axis=1)).ravel()
    Ahat = sp.diags(1.0 / d) @ W
    return d, Ahat.tocsr()


def features(g, e2) -> np.ndarray:
    d, Ahat = graph_ops(g)
    u = normalise(e2)
    ld = np.log(d)
    ld = ld - ld.mean()
    return np.stack([u, Ahat @ u, ld, Ahat @ ld], axis=1).astype(np.float32)


def forward(theta, g, e2, bf=True, dtype=np.float32):
    """Returns y and the cache for backward.  dtype float64 with bf=False is
    the exact function used for finite-difference checks."""
    q = (lambda a: bf16(a)) if bf else (lambda a: a)
    _, Ahat = graph_ops(g)
    Ahat = Ahat.astype(dtype)
    P = [p.astype(dtype) for p in unpack(theta)]
    F = features(g, e2).astype(dtype)
    W0, b0 = P[0], P[1]
    pre = [F @ W0 + b0]
    h = [np.maximum(pre[0], 0)]
    zs = []
    for k in range(LAYERS):
        Wk, bk = P[2 + 2 * k], P[3 + 2 * k]
        z = np.concatenate([h[-1], Ahat @ h[-1]], axis=1).astype(dtype)
        zs.append(z)
        pk = (q(z).astype(dtype) @ q(Wk).astype(dtype)).astype(dtype) + bk
        pre.append(pk)
        h.append(np.maximum(pk, 0))
    wo, bo = P[-2], P[-1]
    u = F[:, 0]
    y = h[-1] @ wo + bo[0] + u
    return y.astype(dtype), dict(F=F, pre=pre, h=h, z=zs, Ahat=Ahat, P=P, bf=bf, dtype=dtype)


def loss(y, t) -> float:
    r = np.asarray(y, np.float64) - normalise(t)
    return 0.5 * float(np.mean(r * r))


def backward(cache, y, t):
    """Gradient of the loss with respect to theta (packed, float64 array)."""
    dtype = cache["dtype"]
    q = (lambda a: bf16(a)) if cache["bf"] else (lambda a: a)
    P, h, pre, zs, F, Ahat = cache["P"], cache["h"], cache["pre"], cache["z"], cache["F"], cache["Ahat"]
    n = len(y)
    dy = ((y.astype(np.float64) - normalise(t)) / n).astype(dtype)
    grads = [None] * len(P)
    grads[-2] = h[-1].T @ dy
    grads[-1] = np.array([dy.sum()], dtype=dtype)
    dh = np.outer(dy, P[-2]).astype(dtype)
    for k in reversed(range(LAYERS)):
        dpre = dh * (pre[k + 1] > 0)
        Wk = P[2 + 2 * k]
        grads[2 + 2 * k] = (q(zs[k]).astype(dtype).T @ q(dpre).astype(dtype)).astype(dtype)
        grads[3 + 2 * k] = dpre.sum(axis=0)
        dz = (q(dpre).astype(dtype) @ q(Wk).astype(dtype).T).astype(dtype)
        dh = dz[:, :HIDDEN] + (Ahat.T @ dz[:, HIDDEN:]).astype(dtype)
    dpre0 = dh * (pre[0] > 0)
    grads[0] = F.T @ dpre0
    grads[1] = dpre0.sum(axis=0)
    return pack(grads)


def loss_and_grad(theta, g, e2, t, bf=True, dtype=np.float32):
    y, cache = forward(theta, g, e2, bf=bf, dtype=dtype)
    return loss(y, t), backward(cache, y, t), y


def adam(theta, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) in float32; step counts from 1."""
    theta = theta.astype(np.float32)
    g = grad.astype(np.float32)
    m = (b1 * m + (1 - b1) * g).astype(np.float32)
    v = (b2 * v + (1 - b2) * g * g).astype(np.float32)
    mh = m / np.float32(1 - b1 ** step)
    vh = v / np.float32(1 - b2 ** step)
    return (theta - np.float32(lr) * mh / (np.sqrt(vh) + np.float32(eps))).astype(np.float32), m, v
