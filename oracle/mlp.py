"""CPU reference of the surrogate network (TEST INFRASTRUCTURE ONLY).

Plain NumPy in float64.  The network is a multilayer perceptron
2 -> 256 -> 256 -> 256 -> 64 with a linear output, trained on mean squared
error with Adam.  Its first layer is a fixed random Fourier-feature map:
a1 = sin(x W1^T + b1), W1 holding 128 random frequency vectors (each twice)
and b1 the phases 0 and pi/2, so that a1 carries the sine and the cosine of
each frequency (Rahimi and Recht, 2007; Tancik et al., 2020); it is not
trained (its gradients are zero).  The two hidden layers after it use GELU.
The paper has no learned component: the architecture, the loss and the
optimiser are this project's definition (the screening of Keller--Miksis
sweeps is the paper's frequency-response study, Sec. 4.2, at higher
resolution).

* GELU(x) = x Phi(x) with the exact Gaussian CDF Phi (Hendrycks and Gimpel,
  "Gaussian Error Linear Units", 2016); GELU'(x) = Phi(x) + x phi(x).
* Adam (Kingma and Ba, 2015): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  w <- w - lr m_hat / (sqrt(v_hat) + eps), with bias corrections
  m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t).
* Parameters are packed in the order W1, b1, W2, b2, W3, b3, W4, b4, each
  weight matrix row-major with shape (out, in): z = a W^T + b.
* Loss: the weighted mean squared error sum_j w_j (out_j - t_j)^2 / (rows x
  outputs), with output 0 (the largest of the targets, which are sorted in
  decreasing order) weighted 32 times the others and the weights scaled to
  mean 1 (OUT_WEIGHTS); with w = None all weights are 1.

``bf16=True`` reproduces the points where the GPU kernels round to bfloat16
(round to nearest, ties to even): the matrix operands of every
matrix-core product (the weights W2..W4 and the activations / gradients that
enter them); everything else stays float64 here.
"""
from __future__ import annotations

import math

import numpy as np

DIMS = (2, 256, 256, 256, 64)
OUT_WEIGHTS = np.r_[32.0, np.ones(63)] * (64.0 / 95.0)


def param_shapes(dims=DIMS):
    shapes = []
    for i in range(len(dims) - 1):
        shapes.append((dims[i + 1], dims[i]))
        shapes.append((dims[i + 1],))
    return shapes


def n_params(dims=DIMS):
    return sum(int(np.prod(s)) for s in param_shapes(dims))


def unpack(flat, dims=DIMS):
    out, o = [], 0
    for s in param_shapes(dims):
        k = int(np.prod(s))
        out.append(np.asarray(flat[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def pack(arrays):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in arrays])


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    r = r.astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def forward(params, x, bf16=False):
    """Returns the output and the cache needed by backward."""
    Ws = params[0::2]
    bs = params[1::2]
    r = bf16_round if bf16 else (lambda a: a)
    a = np.asarray(x, dtype=np.float64)
    cache = {"a": [a], "z": []}
    L = len(Ws)
    for l in range(L):
        W = Ws[l]
        if l == 0:
            z = a @ W.T + bs[l]                      # K = 2: vector unit, no rounding
        else:
            z = r(a) @ r(W).T + bs[l]
        cache["z"].append(z)
        if l == 0:
            a = np.sin(z)                            # the fixed Fourier features
            cache["a"].append(a)
        elif l < L - 1:
            a = gelu(z)
            cache["a"].append(a)
        else:
            a = z
    return a, cache


def mse(out, target, w=None):
    d = out - target
    if w is not None:
        return float(np.mean(np.asarray(w) * d * d))
    return float(np.mean(d * d))


def backward(params, cache, out, target, bf16=False, w=None):
    """Gradients of the mean squared error with respect to every parameter
    (zero for the fixed feature layer W1, b1)."""
    Ws = params[0::2]
    r = bf16_round if bf16 else (lambda a: a)
    L = len(Ws)
    B, O = out.shape
    dz = 2.0 * (out - target) / (B * O)
    if w is not None:
        dz = dz * np.asarray(w)
    grads = [None] * (2 * L)
    grads[0] = np.zeros_like(Ws[0])
    grads[1] = np.zeros(Ws[0].shape[0])
    for l in range(L - 1, 0, -1):
        a_prev = cache["a"][l]
        grads[2 * l] = r(dz).T @ r(a_prev)
        grads[2 * l + 1] = dz.sum(axis=0)
        if l > 1:
            da = r(dz) @ r(Ws[l])
            dz = da * gelu_grad(cache["z"][l - 1])
    return grads


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, fixed=0):
    """One Adam update (t is the 1-based step count); returns new (params, m,
    v).  The first `fixed` arrays (the feature layer's W1, b1: 2) are left
    as they are."""
    out_p, out_m, out_v = [], [], []
    for k, (p, g, mm, vv) in enumerate(zip(params, grads, m, v)):
        if k < fixed:
            out_p.append(p)
            out_m.append(mm)
            out_v.append(vv)
            continue
        mm = b1 * mm + (1.0 - b1) * g
        vv = b2 * vv + (1.0 - b2) * g * g
        mh = mm / (1.0 - b1 ** t)
        vh = vv / (1.0 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v
