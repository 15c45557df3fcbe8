"""Pins of the surrogate-network oracle (NumPy FP64) against mathematics."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from paper_2011_01740_amd import inputs as I

SMALL = (2, 5, 4, 3, 2)


def test_parameter_count_of_the_surrogate():
    assert M.n_params() == 148800
    flat = I.mlp_init(4)
    assert flat.size == 148800
    ps = M.unpack(flat)
    assert [p.shape for p in ps] == M.param_shapes()
    assert np.array_equal(M.pack(ps), flat)
    lim = math.sqrt(6.0 / 256)
    assert np.abs(ps[2]).max() <= lim and np.all(ps[3] == 0)
    # the feature layer: each frequency twice, phases 0 and pi/2
    assert np.array_equal(ps[0][:128], ps[0][128:])
    assert np.all(ps[1][:128] == 0) and np.all(ps[1][128:] == np.pi / 2)
    assert 10 < ps[0].std() < 22


def test_feature_layer_is_sine_and_cosine_of_each_frequency():
    ps = M.unpack(I.mlp_init(4))
    x = np.random.default_rng(3).uniform(-1, 1, size=(50, 2))
    _, cache = M.forward(ps, x)
    a1 = cache["a"][1]
    z = x @ ps[0][:128].T
    assert np.allclose(a1[:, :128], np.sin(z), rtol=0, atol=1e-12)
    assert np.allclose(a1[:, 128:], np.cos(z), rtol=0, atol=1e-12)
    assert np.allclose(a1[:, :128] ** 2 + a1[:, 128:] ** 2, 1.0, atol=1e-12)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000).astype(np.float32) * 10 ** rng.uniform(-20, 20, 5000).astype(np.float32),
                        np.float32([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -1e-40, np.inf, -np.inf])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert M.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert M.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6


def test_gelu_identities():
    x = np.linspace(-8, 8, 1601)
    g = M.gelu(x)
    # Phi(x) + Phi(-x) = 1  =>  GELU(x) - GELU(-x) = x
    assert np.allclose(g - M.gelu(-x), x, rtol=0, atol=1e-14)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert M.gelu_grad(np.array([0.0]))[0] == 0.5
    assert abs(M.gelu(np.array([10.0]))[0] - 10.0) < 1e-20
    assert abs(M.gelu(np.array([-10.0]))[0]) < 1e-20
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(x), fd, atol=1e-8)


def _rand_params(dims, seed):
    rng = np.random.default_rng(seed)
    ps = []
    for i in range(len(dims) - 1):
        ps.append(rng.normal(scale=0.7, size=(dims[i + 1], dims[i])))
        ps.append(rng.normal(scale=0.2, size=dims[i + 1]))
    return ps


@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_matches_central_differences(weighted):
    """Gradients of the trained layers (2 .. 4) against central differences of
    the loss; the fixed feature layer's are zero by definition."""
    rng = np.random.default_rng(1)
    ps = _rand_params(SMALL, 2)
    x = rng.normal(size=(7, 2))
    t = rng.normal(size=(7, 2))
    w = np.array([3.0, 0.5]) if weighted else None
    out, cache = M.forward(ps, x)
    grads = M.backward(ps, cache, out, t, w=w)
    assert np.all(grads[0] == 0) and np.all(grads[1] == 0)
    h = 1e-6
    for k, p in enumerate(ps):
        if k < 2:
            continue
        fd = np.zeros_like(p)
        for idx in np.ndindex(p.shape):
            old = p[idx]
            p[idx] = old + h
            lp = M.mse(M.forward(ps, x)[0], t, w)
            p[idx] = old - h
            lm = M.mse(M.forward(ps, x)[0], t, w)
            p[idx] = old
            fd[idx] = (lp - lm) / (2 * h)
        err = np.abs(grads[k] - fd).max() / max(np.abs(fd).max(), 1e-12)
        assert err < 1e-6, (k, err)


def test_forward_closed_form_tiny_network():
    # one unit per layer: out = w4 * g(g(sin(w1 . x + b1))) - 1
    dims = (2, 1, 1, 1, 1)
    ps = [np.array([[1.0, -2.0]]), np.array([0.5]), np.array([[1.0]]), np.array([0.0]),
          np.array([[1.0]]), np.array([0.0]), np.array([[3.0]]), np.array([-1.0])]
    x = np.array([[0.3, 0.1]])
    z = 0.3 - 0.2 + 0.5
    def g(v):
        return 0.5 * v * (1 + math.erf(v / math.sqrt(2)))
    want = 3.0 * g(g(math.sin(z))) - 1.0
    out, _ = M.forward(ps, x)
    assert out[0, 0] == pytest.approx(want, rel=1e-15)


def test_perfect_fit_has_zero_gradient():
    ps = _rand_params(SMALL, 3)
    x = np.random.default_rng(4).normal(size=(5, 2))
    out, cache = M.forward(ps, x)
    grads = M.backward(ps, cache, out, out.copy())
    assert M.mse(out, out) == 0.0
    assert all(np.all(g == 0) for g in grads)


def test_adam_first_step_is_signed_learning_rate():
    # bias-corrected first moments are g and g^2: the step is lr g / (|g| + eps)
    g = [np.array([3.0, -0.5, 1e-3, 0.0])]
    p = [np.zeros(4)]
    z = [np.zeros(4)]
    p1, m1, v1 = M.adam_step(p, g, z, z, t=1, lr=0.01)
    want = -0.01 * g[0] / (np.abs(g[0]) + 1e-8)
    assert np.allclose(p1[0], want, rtol=1e-12, atol=0)
    assert np.allclose(m1[0], 0.1 * g[0]) and np.allclose(v1[0], 0.001 * g[0] ** 2)


def test_adam_minimises_a_quadratic():
    c = np.array([1.5, -2.0, 0.25])
    p = [np.zeros(3)]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    for t in range(1, 4001):
        g = [2 * (p[0] - c)]
        p, m, v = M.adam_step(p, g, m, v, t, lr=0.01)
    assert np.allclose(p[0], c, atol=1e-3)


def test_bf16_mode_rounds_matrix_operands_only():
    ps = _rand_params(SMALL, 5)
    x = np.random.default_rng(6).normal(size=(4, 2))
    a, _ = M.forward(ps, x)
    b, _ = M.forward(ps, x, bf16=True)
    rel = np.abs(a - b).max() / np.abs(a).max()
    assert 0 < rel < 3e-2
