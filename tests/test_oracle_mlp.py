"""Pins of the surrogate network's FP64 reference (oracle/mlp.py), CPU only.

The gradient is pinned by central finite differences of the loss (FP64, no
rounding); BF16 rounding by torch's own float32 -> bfloat16 conversion and by
hand-checked bit patterns; the conservation projection by its defining
properties.
"""
import numpy as np
import pytest

from oracle import mlp


def small_net(seed, dims):
    rng = np.random.default_rng(seed)
    return [(rng.normal(0, 1 / np.sqrt(i), size=(o, i)), rng.normal(0, 0.1, size=o))
            for i, o in zip(dims[:-1], dims[1:])]


def test_bf16_rounding_bit_patterns():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1)
    assert mlp.to_bf16(1.0 + 2 ** -8) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert mlp.to_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert mlp.to_bf16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
    assert mlp.to_bf16(-2.5) == -2.5
    assert np.isinf(mlp.to_bf16(np.inf))


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).normal(size=20000) * np.exp(np.random.default_rng(1).normal(size=20000) * 5)
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.to_bf16(x), ref)


@pytest.mark.parametrize("relative", [False, True])
def test_gradient_matches_finite_differences(relative):
    dims = [7, 11, 9, 7]
    params = small_net(3, dims)
    rng = np.random.default_rng(4)
    f = rng.normal(size=(5, 7))
    q = rng.normal(size=(5, 7)) * np.array([[1.0], [0.1], [3.0], [1.0], [0.5]])
    mu_in, sd_in = rng.normal(size=7) * 0.1, 1 + rng.random(7)
    mu_out, sd_out = rng.normal(size=7) * 0.1, 1 + rng.random(7)
    kw = dict(bf16=False, relative=relative)
    _, grads = mlp.loss_and_grad(params, f, q, mu_in, sd_in, mu_out, sd_out, **kw)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for (arr, g) in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            for idx in np.random.default_rng(li).choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = mlp.loss_and_grad(params, f, q, mu_in, sd_in, mu_out, sd_out, **kw)
                flat[idx] = old - h
                lm, _ = mlp.loss_and_grad(params, f, q, mu_in, sd_in, mu_out, sd_out, **kw)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g.reshape(-1)[idx]) <= 1e-7 * max(1.0, abs(fd)), (li, idx, fd, g.reshape(-1)[idx])


def test_relative_loss_special_values():
    """With mu_out = 0 a network whose output is zero has relative error 1 for
    every row (loss 1), and one that returns the normalised target exactly has
    loss 0, whatever the row scales and sd_out."""
    dims = [6, 8, 5]
    rng = np.random.default_rng(9)
    f = rng.normal(size=(4, 6))
    q = rng.normal(size=(4, 5)) * np.array([[1e-3], [1.0], [10.0], [0.2]])
    z_in, o_in = np.zeros(6), np.ones(6)
    sd_out = 0.5 + rng.random(5)
    zero = [(np.zeros((o, i)), np.zeros(o)) for i, o in zip(dims[:-1], dims[1:])]
    loss, _ = mlp.loss_and_grad(zero, f, q, z_in, o_in, np.zeros(5), sd_out, bf16=False, relative=True)
    assert abs(loss - 1.0) <= 1e-14
    # a last layer that outputs y = q / sd_out exactly: weights 0, bias per row is impossible,
    # so use one row and put the target in the bias
    W = [(np.zeros((8, 6)), np.zeros(8)), (np.zeros((5, 8)), q[1] / sd_out)]
    loss, _ = mlp.loss_and_grad(W, f[1:2], q[1:2], z_in, o_in, np.zeros(5), sd_out, bf16=False, relative=True)
    assert loss <= 1e-28


def test_bf16_gradient_close_to_fp64():
    """Rounding at the BF16 points moves the gradient by BF16 precision, not more."""
    dims = [16, 32, 32, 16]
    params = small_net(5, dims)
    rng = np.random.default_rng(6)
    f, q = rng.normal(size=(8, 16)), rng.normal(size=(8, 16))
    z, o = np.zeros(16), np.ones(16)
    l64, g64 = mlp.loss_and_grad(params, f, q, z, o, z, o, bf16=False)
    l16, g16 = mlp.loss_and_grad(params, f, q, z, o, z, o, bf16=True)
    assert abs(l16 - l64) <= 2e-2 * l64
    for (a, _), (b, _) in zip(g16, g64):
        assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(b)


def test_conservation_projection():
    rng = np.random.default_rng(7)
    C = rng.normal(size=(3, 20))
    q = rng.normal(size=(4, 20))
    p = mlp.conserve(q, C)
    assert np.max(np.abs(p @ C.T)) <= 1e-12 * np.max(np.abs(q))
    # idempotent, and it only removes the span of the constraints
    assert np.allclose(mlp.conserve(p, C), p, atol=1e-13)
    d = q - p
    coef, *_ = np.linalg.lstsq(C.T, d.T, rcond=None)
    assert np.allclose(C.T @ coef, d.T, atol=1e-12)
