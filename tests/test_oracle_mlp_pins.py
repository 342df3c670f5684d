"""Pins of the FP64 warm-start MLP oracle: central finite differences of the
loss, a self-generated target (zero loss, zero gradient), the output
transform at special values and the first Adam step in closed form."""
import numpy as np
import pytest

from oracle import mlp
from paper_2508_16094_amd import workloads as w


def _net(seed=3, dims=(5, 7, 6, 5)):
    params = w.mlp_init(list(dims), seed)
    rng = np.random.default_rng(seed)
    # non-zero biases so that ReLU kinks are away from the sample points
    params = [(W * 3.0, rng.uniform(-0.5, 0.5, b.shape)) for W, b in params]
    X = rng.standard_normal((4, dims[0]))
    T = np.concatenate([rng.uniform(0.5, 9.5, (4, 3)), rng.uniform(0.01, 5.0, (4, dims[-1] - 3))], axis=1)
    return params, X, T


@pytest.mark.parametrize("xw", [1.0, 7.0])
def test_gradient_matches_central_differences(xw):
    params, X, T = _net()
    loss, grads = mlp.gradients(params, X, T, n_x=3, x_weight=xw)
    assert loss > 0
    worst = 0.0
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            for idx in np.ndindex(arr.shape):
                h = 1e-6 * max(1.0, abs(arr[idx]))
                old = arr[idx]
                arr[idx] = old + h
                fp = mlp.loss_of(params, X, T, 3, x_weight=xw)
                arr[idx] = old - h
                fm = mlp.loss_of(params, X, T, 3, x_weight=xw)
                arr[idx] = old
                fd = (fp - fm) / (2 * h)
                worst = max(worst, abs(fd - g[idx]) / max(1e-3, abs(fd), abs(g[idx])))
    assert worst <= 1e-6, worst


def test_self_generated_target_has_zero_loss_and_gradient():
    params, X, _ = _net(seed=5)
    _, z = mlp.forward(params, X)
    T = mlp.transform(z, 3)
    loss, grads = mlp.gradients(params, X, T, n_x=3)
    assert loss <= 1e-20
    assert max(np.abs(g).max() for gw in grads for g in gw) <= 1e-10


def test_output_transform_special_values():
    z = np.array([[0.0, 0.0, 40.0, -40.0, 0.0]])
    out = mlp.transform(z, 2, x_scale=10.0)
    assert np.allclose(out[0, :2], [5.0, 5.0])
    assert abs(out[0, 2] - 40.0) < 1e-12          # softplus(40) = 40 + log1p(e^-40)
    assert 0 < out[0, 3] < 1e-17                   # softplus(-40) = e^-40 (to first order)
    assert abs(out[0, 4] - np.log(2.0)) < 1e-15


def test_first_adam_step_closed_form():
    params, X, T = _net(seed=7)
    _, grads = mlp.gradients(params, X, T, n_x=3)
    opt = mlp.Adam(params)
    lr = 1e-3
    new = opt.step(params, grads, lr)
    for (W, b), (gW, gb), (W1, b1) in zip(params, grads, new):
        # m_hat = g, v_hat = g^2 after one step: p - lr g / (|g| + eps)
        assert np.allclose(W1, W - lr * gW / (np.abs(gW) + 1e-8), rtol=0, atol=1e-15)
        assert np.allclose(b1, b - lr * gb / (np.abs(gb) + 1e-8), rtol=0, atol=1e-15)


def test_training_reduces_loss():
    params, X, T = _net(seed=9)
    opt = mlp.Adam(params)
    l0 = mlp.loss_of(params, X, T, 3)
    for _ in range(200):
        _, g = mlp.gradients(params, X, T, 3)
        params = opt.step(params, g, 1e-2)
    assert mlp.loss_of(params, X, T, 3) < 0.2 * l0


def test_gradient_magnitudes_bound_the_gradients():
    """Each magnitude is a sum of absolute values of the gradient's own terms
    (over a superset of the active units): it bounds |gradient| entry by
    entry, with equality when every term has one sign."""
    from paper_2508_16094_amd import workloads as w
    dims = [8, 32, 24, 20]
    params = w.mlp_init(dims, 5)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((17, 8))
    T = np.concatenate([rng.uniform(1, 9, (17, 12)), rng.uniform(0.1, 2, (17, 8))], axis=1)
    _, g = mlp.gradients(params, X, T, 12)
    mags = mlp.gradient_magnitudes(params, X, T, 12)
    for (gW, gb), (mW, mb) in zip(g, mags):
        assert np.all(np.abs(gW) <= mW * (1 + 1e-12) + 1e-300)
        assert np.all(np.abs(gb) <= mb * (1 + 1e-12) + 1e-300)
    # a batch of one with one output: every term of the last layer's weight
    # gradient is a single product, so magnitude = |gradient|
    one = [(rng.standard_normal((1, 8)), np.zeros(1))]
    _, g1 = mlp.gradients(one, np.abs(X[:1]), T[:1, :1], 1)
    m1 = mlp.gradient_magnitudes(one, np.abs(X[:1]), T[:1, :1], 1)
    assert np.allclose(np.abs(g1[0][0]), m1[0][0], rtol=1e-14)
