"""Pins of the reference network of the learned extension (oracle/mpnn.py):
bf16 rounding against an independent construction, analytic gradients
against central differences, invariances, and the Adam closed form."""
import numpy as np
import pytest

from oracle import mpnn as M
from paper_1806_07028_amd import inputs as I


def bf16_by_frexp(x):
    """Nearest bfloat16 (8 significant bits, ties to even) via frexp/rint."""
    x = np.asarray(x, dtype=np.float64)
    mant, ex = np.frexp(x)            # x = mant * 2^ex, 0.5 <= |mant| < 1
    return (np.rint(mant * 256.0) / 256.0 * np.exp2(ex)).astype(np.float32)


def test_bf16_rounding():
    special = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7 + 2 ** -8, -1.5 - 2 ** -9,
                        3.14159265, 1e-20, -7.25e10, 0.0], dtype=np.float32)
    got = M.bf16(special)
    assert got[0] == 1.0 and got[1] == 1.0                      # halfway: ties to even (down)
    assert got[2] == np.float32(1.0 + 2 ** -7)                   # above halfway: up
    assert got[3] == np.float32(1.0 + 2 ** -6)                   # halfway, odd below: up to even
    rnd = np.random.default_rng(0).standard_normal(4000).astype(np.float32) * np.float32(1e3)
    x = np.concatenate([special, rnd])
    assert np.array_equal(M.bf16(x), bf16_by_frexp(x))


@pytest.fixture(scope="module")
def small():
    g = I.rgg(80, 5)
    n = g[0]
    e2 = I.normal(3, n)
    t = I.normal(4, n) + 0.5 * e2
    return g, e2, t


def test_gradient_matches_central_differences(small):
    g, e2, t = small
    theta = M.init_params(1).astype(np.float64)
    rng = np.random.default_rng(2)
    theta[M.NFEAT * M.HIDDEN:M.NFEAT * M.HIDDEN + M.HIDDEN] = rng.uniform(0.05, 0.2, M.HIDDEN)  # live ReLUs
    f = lambda th: M.loss(M.forward(th, g, e2, bf=False, dtype=np.float64)[0], t)
    L, grad, _ = M.loss_and_grad(theta, g, e2, t, bf=False, dtype=np.float64)
    assert abs(L - f(theta)) < 1e-15
    idx = np.concatenate([rng.choice(M.NPARAMS, 120, replace=False), [M.NPARAMS - 1, M.NPARAMS - 2, 0]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (f(tp) - f(tm)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, grad[i])


def test_invariances_and_precision(small):
    g, e2, t = small
    theta = M.init_params(3)
    y1, _ = M.forward(theta, g, e2, bf=False)
    y2, _ = M.forward(theta, g, 3.0 * e2 + 5.0, bf=False)
    assert np.allclose(y1, y2, rtol=0, atol=1e-5)
    yb, _ = M.forward(theta, g, e2, bf=True)
    assert np.linalg.norm(yb - y1) <= 2e-2 * np.linalg.norm(y1)
    # the output is u plus the network's correction: zero output weights give u
    th0 = theta.copy()
    th0[-M.HIDDEN - 1:] = 0
    y0, cache = M.forward(th0, g, e2)
    assert np.allclose(y0, M.normalise(e2), atol=1e-6)
    assert M.loss(y0, t) == pytest.approx(0.5 * np.mean((M.normalise(e2) - M.normalise(t)) ** 2), rel=1e-6)


def test_adam_first_step_is_signed_lr():
    theta = np.linspace(-1, 1, 11).astype(np.float32)
    grad = np.array([3, -2, 1e-3, -5e-3, 7, 0.5, -0.5, 2, -2, 1, -1], dtype=np.float64)
    out, m, v = M.adam(theta, np.zeros(11, np.float32), np.zeros(11, np.float32), grad, 1, 0.01)
    assert np.allclose(out, theta - 0.01 * np.sign(grad), atol=1e-6)
