"""GPU warm-start MLP (BF16 MFMA products, FP32 accumulation) against the
FP64 oracle MLP.

Bars: outputs within 1e-2 (1 + |ref|) of the oracle evaluated with the same
BF16-rounded parameters and inputs (the GPU also rounds hidden activations
to BF16); loss within 2e-2 relative; gradient cosine >= 0.99 for every
weight matrix and bias; the first Adam step equals its closed form on the
GPU's own gradients (FP32, 1e-6 absolute)."""
import numpy as np
import pytest

from _util import bf16_round
from oracle import mlp as omlp
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DIMS = [16, 64, 48, 70]
NX = 40


def _setup(seed=1, B=33):
    params = w.mlp_init(DIMS, seed)
    rng = np.random.default_rng(seed)
    params = [(W, rng.uniform(-0.2, 0.2, b.shape)) for W, b in params]
    X = rng.standard_normal((B, DIMS[0]))
    T = np.concatenate([rng.uniform(0.5, 9.5, (B, NX)), rng.uniform(0.01, 3.0, (B, DIMS[-1] - NX))], axis=1)
    return params, X, T


def _bf16_params(params):
    return [(bf16_round(W), b.astype(np.float32).astype(np.float64)) for W, b in params]


def _model(params, max_batch=64, x_weight=1.0):
    m = L.MlpModel(DIMS, NX, max_batch=max_batch, x_weight=x_weight).bind()
    m.set_params(params)
    return m


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device="cuda:0")


@pytest.mark.parametrize("B", [1, 33, 64])
def test_mlp_forward_matches_oracle(B):
    params, X, _ = _setup(B=B)
    m = _model(params)
    out = m.forward(_dev(X)).cpu().numpy().astype(np.float64)
    _, z = omlp.forward(_bf16_params(params), bf16_round(X))
    ref = omlp.transform(z, NX)
    assert np.all(np.abs(out - ref) <= 1e-2 * (1 + np.abs(ref))), np.max(np.abs(out - ref))


@pytest.mark.parametrize("xw", [1.0, 50.0])
def test_mlp_gradients_match_oracle(xw):
    params, X, T = _setup(seed=2, B=48)
    m = _model(params, x_weight=xw)
    loss, grads = m.gradients(_dev(X), _dev(T))
    lref, gref = omlp.gradients(_bf16_params(params), bf16_round(X), T, NX, x_weight=xw)
    assert abs(loss - lref) <= 2e-2 * lref, (loss, lref)
    for (gW, gb), (rW, rb) in zip(grads, gref):
        for a, r in ((gW, rW), (gb, rb)):
            a = a.astype(np.float64).ravel(); r = r.ravel()
            cos = a @ r / (np.linalg.norm(a) * np.linalg.norm(r) + 1e-300)
            assert cos >= 0.99, cos


def test_mlp_first_adam_step_and_training():
    params, X, T = _setup(seed=3, B=40)
    m = _model(params)
    p0 = m.get_params()
    _, g = m.gradients(_dev(X), _dev(T))
    lr = 1e-3
    l0 = m.train_step(_dev(X), _dev(T), lr)
    p1 = m.get_params()
    for (W0, b0), (gW, gb), (W1, b1) in zip(p0, g, p1):
        assert np.allclose(W1, W0 - lr * gW / (np.abs(gW) + 1e-8), rtol=0, atol=1e-6)
        assert np.allclose(b1, b0 - lr * gb / (np.abs(gb) + 1e-8), rtol=0, atol=1e-6)
    for _ in range(150):
        last = m.train_step(_dev(X), _dev(T), 3e-3)
    assert last < 0.3 * l0, (l0, last)


def test_mlp_deterministic_and_errors():
    params, X, T = _setup(seed=4, B=20)
    m = _model(params, max_batch=32)
    a = m.forward(_dev(X)).cpu().numpy()
    b = m.forward(_dev(X)).cpu().numpy()
    assert np.array_equal(a, b)
    la, ga = m.gradients(_dev(X), _dev(T))
    lb, gb = m.gradients(_dev(X), _dev(T))
    assert la == lb and all(np.array_equal(x[0], y[0]) for x, y in zip(ga, gb))
    with pytest.raises(L.PdipmError) as e:
        m.forward(_dev(np.zeros((33, DIMS[0]))))
    assert e.value.code == L.PDIPM_ERR_INVALID_ARG


@pytest.mark.parametrize("B", [256, 512])
def test_mlp_gradients_elementwise_at_production_shapes(B):
    """64 -> 512 -> 512 -> 4096 (the production net's layer shapes with a
    narrower output): the K = 512 products of the forward pass and the
    K = 4096 product of the last layer's backward pass run split-K, and so do
    the weight gradients (K = B) at B = 512.  Every gradient entry is within
    16 u_bf16 (u_bf16 = 2^-8) of the FP64 oracle's, relative to the sum of
    the absolute values of its terms (the rounding-error scale of a dot
    product whose factors are rounded to BF16; 16 covers the roundings of
    the three layers' inputs and of dL/dz)."""
    dims = [64, 512, 512, 4096]
    nx = 2731
    params = w.mlp_init(dims, 11)
    rng = np.random.default_rng(12)
    params = [(W, rng.uniform(-0.1, 0.1, b.shape)) for W, b in params]
    X = rng.standard_normal((B, dims[0]))
    T = np.concatenate([rng.uniform(0.5, 9.5, (B, nx)), rng.uniform(0.01, 3.0, (B, dims[-1] - nx))], axis=1)
    print(f"case mlp gradients production shapes B={B}", flush=True)
    m = L.MlpModel(dims, nx, max_batch=B, x_weight=1e4).bind()
    m.set_params(params)
    loss, grads = m.gradients(_dev(X), _dev(T))
    pb, Xb = _bf16_params(params), bf16_round(X)
    lref, gref = omlp.gradients(pb, Xb, T, nx, x_weight=1e4)
    mags = omlp.gradient_magnitudes(pb, Xb, T, nx, x_weight=1e4)
    assert abs(loss - lref) <= 2e-2 * lref, (loss, lref)
    bound = 16 * 2.0 ** -8
    worst = 0.0
    for (gW, gb), (rW, rb), (mW, mb) in zip(grads, gref, mags):
        for a, r, mg in ((gW, rW, mW), (gb, rb, mb)):
            err = np.abs(a.astype(np.float64) - r)
            assert np.all(err <= bound * mg + 1e-30), np.max(err / (mg + 1e-300))
            worst = max(worst, float(np.max(err / (mg + 1e-300))))
    print(f"worst |g - g_ref| / magnitude = {worst:.3e} (bound {bound:.3e})", flush=True)
