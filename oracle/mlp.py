"""FP64 reference of the surrogate network -- test infrastructure only.

The learned surrogate of the reaction M2L integrals (an alternative to the
quadrature of Section 3.5, standing where the paper uses pre-computed tables) is a
multilayer perceptron: ``H`` hidden layers of width ``W`` with the SiLU activation
silu(z) = z / (1 + e^{-z}) and a linear output layer, trained on the mean squared
error with Adam (Kingma & Ba, 2015).  This module computes the forward pass, the
gradients by a backward pass written out by hand (chain rule, layer by layer) and
one Adam step, in plain numpy FP64.

``mimic=True`` rounds to bfloat16 (round to nearest, ties to even, from float32) at
the points where the GPU kernels hold BF16 operands: the network input, the weights,
the hidden activations, the output gradient and the pre-activation gradients.  All
arithmetic between those points stays FP64 here.

Only ``tests/`` may import this module.  Pins (``tests/test_oracle_mlp.py``): the
backward pass against central finite differences of the forward pass; the BF16
rounding against exactly representable cases; Adam's first step against its closed
form; training on a target the network can represent drives the loss down.

Parameter packing (the same as the library's): for each layer in order, the weight
matrix row-major [out][in], then the bias [out].
"""
import numpy as np


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), via float32; returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def layer_dims(nin, width, nhidden, nout):
    dims = [nin] + [width] * nhidden + [nout]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def unpack(params, nin, width, nhidden, nout):
    """Split the flat parameter vector into [(W, b)] (views)."""
    out, off = [], 0
    params = np.asarray(params, dtype=np.float64)
    for (o, i) in layer_dims(nin, width, nhidden, nout):
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((W, b))
    assert off == params.size
    return out


def n_params(nin, width, nhidden, nout):
    return sum(o * i + o for (o, i) in layer_dims(nin, width, nhidden, nout))


def init_params(nin, width, nhidden, nout, rng):
    """He-style uniform initialisation, zero biases (the library draws its own)."""
    parts = []
    for (o, i) in layer_dims(nin, width, nhidden, nout):
        lim = np.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def forward(params, x, nin, width, nhidden, nout, mimic=False):
    """Network output y [B, nout] and the saved (pre-activation, activation) pairs."""
    rnd = bf16_round if mimic else (lambda v: v)
    layers = unpack(params, nin, width, nhidden, nout)
    a = rnd(np.asarray(x, dtype=np.float64))
    saved = [(None, a)]
    for li, (W, b) in enumerate(layers):
        z = a @ rnd(W).T + b
        if li == len(layers) - 1:
            return z, saved
        a = rnd(silu(z))
        saved.append((z, a))


def loss_and_grad(params, x, t, nin, width, nhidden, nout, mimic=False):
    """Mean squared error over batch and outputs, its gradient (flat, same packing
    as the parameters) and the network output."""
    rnd = bf16_round if mimic else (lambda v: v)
    layers = unpack(params, nin, width, nhidden, nout)
    y, saved = forward(params, x, nin, width, nhidden, nout, mimic)
    B = y.shape[0]
    r = y - t
    loss = float(np.sum(r * r) / (B * nout))
    d = rnd(2.0 * r / (B * nout))  # dL/dz of the output layer
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a_in = saved[li][1]
        gW = d.T @ a_in
        gb = d.sum(axis=0)
        grads[li] = (gW, gb)
        if li == 0:
            break
        da = d @ rnd(W)
        z_in = saved[li][0]
        d = rnd(da * dsilu(z_in))
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1]]) for g in grads])
    return loss, flat, y


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
