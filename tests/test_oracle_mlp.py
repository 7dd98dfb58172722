"""Pins of the surrogate network's FP64 reference (oracle/mlp.py), CPU only."""
import numpy as np
import pytest

from oracle import mlp

DIMS = dict(nin=6, width=8, nhidden=3, nout=5)


def _setup(seed=0, B=7):
    rng = np.random.default_rng(seed)
    P = mlp.init_params(rng=rng, **DIMS)
    P = P + 0.05 * rng.standard_normal(P.size)  # non-zero biases too
    x = rng.uniform(-1, 1, (B, DIMS["nin"]))
    t = rng.standard_normal((B, DIMS["nout"]))
    return P, x, t


def test_backward_matches_central_differences():
    P, x, t = _setup()
    loss, g, _ = mlp.loss_and_grad(P, x, t, **DIMS)
    h = 1e-6
    rng = np.random.default_rng(1)
    idx = rng.choice(P.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(P)
        e[i] = h
        lp = mlp.loss_and_grad(P + e, x, t, **DIMS)[0]
        lm = mlp.loss_and_grad(P - e, x, t, **DIMS)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_backward_covers_every_layer():
    # a dropped layer or transposed operand would leave some gradient block at 0
    P, x, t = _setup(seed=3)
    _, g, _ = mlp.loss_and_grad(P, x, t, **DIMS)
    off = 0
    for (o, i) in mlp.layer_dims(**DIMS):
        assert np.abs(g[off:off + o * i]).max() > 0
        off += o * i + o


def test_silu_values():
    assert mlp.silu(0.0) == 0.0
    assert mlp.dsilu(0.0) == 0.5
    assert abs(mlp.silu(40.0) - 40.0) < 1e-12
    assert abs(mlp.silu(-40.0)) < 1e-15
    z = np.linspace(-5, 5, 41)
    fd = (mlp.silu(z + 1e-6) - mlp.silu(z - 1e-6)) / 2e-6
    assert np.allclose(fd, mlp.dsilu(z), atol=1e-9)


def test_bf16_round_exact_cases():
    ulp = 2.0 ** -7  # spacing of bfloat16 just above 1
    cases = {1.0: 1.0, 1 + ulp: 1 + ulp, 1 + ulp / 2: 1.0,  # tie -> even mantissa
             1 + 1.5 * ulp: 1 + 2 * ulp,                    # tie -> even mantissa
             1 + 0.75 * ulp: 1 + ulp, -3.0: -3.0, 0.0: 0.0}
    for x, want in cases.items():
        assert mlp.bf16_round(np.array([x]))[0] == want, x
    # unit roundoff of an 8-significant-bit format: 2^-8 (plus the float32 step)
    x = np.random.default_rng(0).uniform(-100, 100, 1000)
    assert np.all(np.abs(mlp.bf16_round(x) - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    p0 = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = mlp.adam_step(p0, g, np.zeros(10), np.zeros(10), 1, lr=1e-2, eps=0.0)
    # bias-corrected moments are g and g^2 after one step: the update is lr * sign(g)
    assert np.allclose(p1, p0 - 1e-2 * np.sign(g), atol=1e-15)


def test_training_reduces_loss_on_representable_target():
    rng = np.random.default_rng(4)
    teacher = mlp.init_params(rng=rng, **DIMS)
    x = rng.uniform(-1, 1, (64, DIMS["nin"]))
    t, _ = mlp.forward(teacher, x, **DIMS)
    P = mlp.init_params(rng=np.random.default_rng(5), **DIMS)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    l0 = mlp.loss_and_grad(P, x, t, **DIMS)[0]
    for s in range(1, 601):
        l, g, _ = mlp.loss_and_grad(P, x, t, **DIMS)
        P, m, v = mlp.adam_step(P, g, m, v, s, lr=1e-2)
    assert l < 1e-2 * l0


@pytest.mark.parametrize("mimic", [False, True])
def test_mimic_only_rounds(mimic):
    # with BF16 rounding the result stays within the rounding level of the FP64 one
    P, x, t = _setup(seed=6)
    y64, _ = mlp.forward(P, x, **DIMS)
    y, _ = mlp.forward(P, x, mimic=mimic, **DIMS)
    rel = np.linalg.norm(y - y64) / np.linalg.norm(y64)
    assert rel < (3e-2 if mimic else 1e-15)
