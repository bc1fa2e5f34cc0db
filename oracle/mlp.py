"""Loop surrogate: multilayer perceptron in plain FP64 (oracle; test infrastructure).

The surrogate maps one compact loop block -- the n_o^4 complex entries of
Lc(q)[dR] of one channel at scale Lambda -- to a fixed feature vector of
(q, Lambda, channel, dR).  The paper has no learned component; this is the
definition the GPU kernels are checked against, written as directly as
possible:

* features of a block (q = 2 pi (mx, my) / Lq on the coarse mesh, channel c,
  difference vector index iD of nD):
    [sin qx, cos qx, sin qy, cos qy, sin 2qx, cos 2qx, sin 2qy, cos 2qy,
     ln(Lambda) / 5, c == 0, c == 1, one-hot(iD)]       (11 + nD values)
* target: Lc(q)[dR] / s(Lambda), real and imaginary parts interleaved in the
  compact entry order (2 n_o^4 values), with s(Lambda) a positive scale table
  interpolated linearly in (ln Lambda, ln s) and constant beyond its ends;
* network: affine layers with GELU(x) = x Phi(x) (Phi the standard normal
  distribution function) after every layer but the last;
* loss: mean of squared errors over batch and outputs;
* optimiser: Adam with bias correction.

Parameters are one flat vector: per layer W[out][in] row-major, then b[out].
"""

import math

import numpy as np

N_FIXED_FEATURES = 11


def features(q_idx, Lq, lam, ch, iD, nD):
    """Feature rows of blocks given by equal-length integer/float arrays."""
    q_idx = np.asarray(q_idx)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), q_idx.shape)
    ch = np.broadcast_to(np.asarray(ch), q_idx.shape)
    iD = np.broadcast_to(np.asarray(iD), q_idx.shape)
    n = q_idx.size
    X = np.zeros((n, N_FIXED_FEATURES + nD))
    qx = 2.0 * np.pi * (q_idx // Lq) / Lq
    qy = 2.0 * np.pi * (q_idx % Lq) / Lq
    X[:, 0] = np.sin(qx)
    X[:, 1] = np.cos(qx)
    X[:, 2] = np.sin(qy)
    X[:, 3] = np.cos(qy)
    X[:, 4] = np.sin(2 * qx)
    X[:, 5] = np.cos(2 * qx)
    X[:, 6] = np.sin(2 * qy)
    X[:, 7] = np.cos(2 * qy)
    X[:, 8] = np.log(lam) / 5.0
    X[np.arange(n), 9 + ch] = 1.0
    X[np.arange(n), N_FIXED_FEATURES + iD] = 1.0
    return X


def scale_interp(lam, lam_tab, s_tab):
    """s(Lambda) from the table: piecewise linear in (ln Lambda, ln s)."""
    x = np.log(np.asarray(lam_tab, dtype=np.float64))
    y = np.log(np.asarray(s_tab, dtype=np.float64))
    o = np.argsort(x)
    return np.exp(np.interp(np.log(lam), x[o], y[o]))


def unpack(params, sizes):
    """List of (W, b) views of the flat parameter vector."""
    params = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for n_i, n_o in zip(sizes[:-1], sizes[1:]):
        W = params[o:o + n_i * n_o].reshape(n_o, n_i)
        o += n_i * n_o
        b = params[o:o + n_o]
        o += n_o
        out.append((W, b))
    assert o == params.size
    return out


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_deriv(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + _erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def _erf(x):
    return np.vectorize(math.erf, otypes=[np.float64])(x)


def forward(params, sizes, X):
    """Network output and the pre-activations of every layer."""
    layers = unpack(params, sizes)
    a = np.asarray(X, dtype=np.float64)
    acts, pre = [a], []
    for i, (W, b) in enumerate(layers):
        z = a @ W.T + b
        pre.append(z)
        a = gelu(z) if i + 1 < len(layers) else z
        acts.append(a)
    return a, acts, pre


def loss(params, sizes, X, T):
    Y, _, _ = forward(params, sizes, X)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def loss_and_grad(params, sizes, X, T):
    """Loss and its gradient with respect to the flat parameter vector
    (reverse-mode chain rule through the affine layers and GELU)."""
    layers = unpack(params, sizes)
    Y, acts, pre = forward(params, sizes, X)
    T = np.asarray(T, dtype=np.float64)
    n, n_out = Y.shape
    L = float(np.mean((Y - T) ** 2))
    d = 2.0 * (Y - T) / (n * n_out)  # dL/dz of the last layer
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        if i + 1 < len(layers):
            d = d * gelu_deriv(pre[i])
        gW = d.T @ acts[i]
        gb = d.sum(axis=0)
        grads.append((gW, gb))
        d = d @ W
    g = []
    for gW, gb in reversed(grads):
        g.append(gW.ravel())
        g.append(gb)
    return L, np.concatenate(g)


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new params, m, v."""
    params = np.asarray(params, dtype=np.float64)
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
