"""Learned warm start: FP64 reference MLP (test infrastructure only).

The paper does not describe a learned warm start; this is the warm-start
form of the benchmark configuration (a parametric QP whose right-hand side
depends on theta): a ReLU multilayer perceptron maps theta to an
interior-point start (x, lambda).  Everything here is plain FP64 numpy in
the order a reader would write it:

  h_0 = theta,  h_l = relu(W_l h_{l-1} + b_l)  (hidden layers),
  z = W_L h_{L-1} + b_L,
  x_hat = x_scale * sigmoid(z[:n_x]),  lambda_hat = softplus(z[n_x:]),
  loss = w_x * mean over batch and x outputs of (sigmoid(z_x) - x / x_scale)^2
       + mean over batch and lambda outputs of
         (log(softplus(z_l) + eps) - log(lambda + eps))^2,   eps = 1e-6.

Parameters are a list of (W, b) with W of shape (out, in); inputs are rows
(batch x features).  The optimiser is Adam with bias correction.
"""
import numpy as np

EPS = 1e-6


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def softplus(z):
    return np.logaddexp(0.0, z)


def forward(params, X):
    """Activations [h_0 .. h_{L-1}] and the output pre-activation z."""
    hs = [np.asarray(X, np.float64)]
    for W, b in params[:-1]:
        hs.append(np.maximum(hs[-1] @ W.T + b, 0.0))
    W, b = params[-1]
    return hs, hs[-1] @ W.T + b


def transform(z, n_x, x_scale=10.0):
    return np.concatenate([x_scale * sigmoid(z[:, :n_x]), softplus(z[:, n_x:])], axis=1)


def loss_and_dz(z, target, n_x, x_scale=10.0, x_weight=1.0):
    """Loss and its gradient with respect to z (target: raw x and lambda)."""
    B = z.shape[0]
    zx, zl = z[:, :n_x], z[:, n_x:]
    tx, tl = target[:, :n_x] / x_scale, np.log(target[:, n_x:] + EPS)
    sx = sigmoid(zx)
    sp = softplus(zl)
    ex = sx - tx
    el = np.log(sp + EPS) - tl
    nx, nl = ex.size, el.size
    loss = (x_weight * np.sum(ex * ex) / nx if nx else 0.0) + (np.sum(el * el) / nl if nl else 0.0)
    dz = np.empty_like(z)
    if nx:
        dz[:, :n_x] = 2.0 * x_weight / nx * ex * sx * (1.0 - sx)
    if nl:
        dz[:, n_x:] = 2.0 / nl * el / (sp + EPS) * sigmoid(zl)
    return loss, dz


def backward(params, hs, dz):
    """Gradients [(dW, db)] of the loss given dL/dz."""
    grads = [None] * len(params)
    d = dz
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        h = hs[l]
        grads[l] = (d.T @ h, d.sum(axis=0))
        if l > 0:
            d = (d @ W) * (h > 0)
    return grads


def loss_of(params, X, target, n_x, x_scale=10.0, x_weight=1.0):
    _, z = forward(params, X)
    return loss_and_dz(z, target, n_x, x_scale, x_weight)[0]


def gradients(params, X, target, n_x, x_scale=10.0, x_weight=1.0):
    hs, z = forward(params, X)
    loss, dz = loss_and_dz(z, target, n_x, x_scale, x_weight)
    return loss, backward(params, hs, dz)


def gradient_magnitudes(params, X, target, n_x, x_scale=10.0, x_weight=1.0, band=2.0 ** -6):
    """For every gradient entry, the sum of the absolute values of the terms
    that make it up (|dL/dz|' |h| propagated back with |W|), the scale
    against which a lower-precision evaluation is judged entry by entry.
    A unit counts as active, and its activation as max(pre + band * |pre|_1, 0),
    when its pre-activation lies within band times the sum of the absolute
    values of its own terms (|W| |h| + |b|) above zero, so that units a
    rounded evaluation may see on either side of the ReLU are included."""
    hs, relaxed = [np.asarray(X, np.float64)], [np.abs(np.asarray(X, np.float64))]
    keeps = []
    for W, b in params[:-1]:
        pre = hs[-1] @ W.T + b
        scale = relaxed[-1] @ np.abs(W).T + np.abs(b)
        keep = pre + band * scale > 0
        keeps.append(keep)
        hs.append(np.maximum(pre, 0.0))
        relaxed.append(np.where(keep, np.abs(pre) + band * scale, 0.0))
    W, b = params[-1]
    z = hs[-1] @ W.T + b
    _, dz = loss_and_dz(z, target, n_x, x_scale, x_weight)
    mags = [None] * len(params)
    d = np.abs(dz)
    for l in range(len(params) - 1, -1, -1):
        Wl, _ = params[l]
        mags[l] = (d.T @ relaxed[l], d.sum(axis=0))
        if l > 0:
            d = (d @ np.abs(Wl)) * keeps[l - 1]
    return mags


class Adam:
    """Adam with bias correction (beta1, beta2, eps as in the usual setting)."""

    def __init__(self, params, beta1=0.9, beta2=0.999, eps=1e-8):
        self.b1, self.b2, self.eps = beta1, beta2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads, lr):
        self.t += 1
        out = []
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            mv = []
            for p, g, m, v in ((W, gW, self.m[i][0], self.v[i][0]), (b, gb, self.m[i][1], self.v[i][1])):
                m = self.b1 * m + (1.0 - self.b1) * g
                v = self.b2 * v + (1.0 - self.b2) * g * g
                new.append(p - lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
                mv.append((m, v))
            self.m[i] = (mv[0][0], mv[1][0])
            self.v[i] = (mv[0][1], mv[1][1])
            out.append((new[0], new[1]))
        return out
