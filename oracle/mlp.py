"""Float64 reference of the learned body-mobility network (spec extension of Sec. 3.1).

The block preconditioner of Sec. 3.1 needs, per rigid body, the body mobility
N~_p = [K_p^T (M^(pp))^-1 K_p]^-1.  Above a wall it depends on the body's
height and orientation only (the wall is invariant under in-plane shifts).
The network maps features of one body to the 21 entries of the lower-triangular
Cholesky factor L of the scaled mobility S = D N~_p D, D = diag(sqrt(6 pi eta a) I3,
sqrt(8 pi eta a^3) I3), so that N~_p = D^-1 L L^T D^-1 is symmetric positive
definite by construction.

Readings (the extension fixes only "height and orientation -> Cholesky factor",
sizes 7 -> 128 -> 128 -> 21 and BF16/FP32 arithmetic):
  * features x = [h/a, s, p1, p2, p3, onehot(type 0), onehot(type 1)] with the
    quaternion sign chosen so that s >= 0 (theta and -theta are one rotation);
  * the 21 outputs are the row-major lower triangle of L with the six diagonal
    entries replaced by their logarithms (L_ii = exp(y) > 0 by construction);
  * inputs and outputs are standardised, x' = (x - mu_x)/sd_x and
    y = mu_y + sd_y * (network output), with constants taken from the training
    set (identity by default), so that every output is learned to a similar
    relative accuracy;
  * hidden activation SiLU, z * sigmoid(z); linear output;
  * loss: mean squared error of the standardised outputs over the 21 outputs
    and the batch;
  * Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the weights; initial weights
    are inputs (drawn by the caller).
"""
from __future__ import annotations

import numpy as np

SIZES = (7, 128, 128, 21)
TRIL = np.tril_indices(6)


def n_params(sizes=SIZES):
    return sum(sizes[i + 1] * sizes[i] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(flat, sizes=SIZES):
    """Flat parameter vector -> [(W (out x in), b (out,)), ...] in layer order."""
    out, k = [], 0
    for i in range(len(sizes) - 1):
        nin, nout = sizes[i], sizes[i + 1]
        W = np.asarray(flat[k:k + nout * nin], float).reshape(nout, nin)
        k += nout * nin
        b = np.asarray(flat[k:k + nout], float)
        k += nout
        out.append((W, b))
    return out


def pack(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def features(height, theta, body_type, a=1.0):
    theta = np.array(theta, float).reshape(-1, 4)
    sgn = np.where(theta[:, 0] < 0, -1.0, 1.0)
    th = theta * sgn[:, None]
    bt = np.asarray(body_type).ravel()
    oh = np.stack([(bt == 0).astype(float), (bt == 1).astype(float)], 1)
    return np.column_stack([np.asarray(height, float).ravel() / a, th, oh])


def scaling(a=1.0, eta=1.0):
    return np.concatenate([np.full(3, np.sqrt(6 * np.pi * eta * a)),
                           np.full(3, np.sqrt(8 * np.pi * eta * a ** 3))])


DIAG = np.where(TRIL[0] == TRIL[1])[0]        # positions of L_ii among the 21


def target_from_mobility(Nt, a=1.0, eta=1.0):
    """21 labels per (6,6) N~: lower triangle of chol(D N~ D), log on the diagonal."""
    d = scaling(a, eta)
    Nt = np.asarray(Nt, float).reshape(-1, 6, 6)
    S = d[None, :, None] * Nt * d[None, None, :]
    L = np.linalg.cholesky(0.5 * (S + S.transpose(0, 2, 1)))
    y = L[:, TRIL[0], TRIL[1]]
    y[:, DIAG] = np.log(y[:, DIAG])
    return y


def mobility_from_output(y, a=1.0, eta=1.0):
    d = scaling(a, eta)
    y = np.array(y, float).reshape(-1, 21)
    y[:, DIAG] = np.exp(y[:, DIAG])
    L = np.zeros((len(y), 6, 6))
    L[:, TRIL[0], TRIL[1]] = y
    S = L @ L.transpose(0, 2, 1)
    return S / d[None, :, None] / d[None, None, :]


def predict(flat, X, mu_x=None, sd_x=None, mu_y=None, sd_y=None, sizes=SIZES):
    """Standardise inputs, run the network, undo the output standardisation."""
    X = np.asarray(X, float)
    Xs = X if mu_x is None else (X - mu_x) / sd_x
    Y, _ = forward(flat, Xs, sizes)
    return Y if mu_y is None else mu_y + sd_y * Y


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(flat, X, sizes=SIZES):
    """Returns (Y, cache).  Hidden layers use SiLU, the last layer is linear."""
    params = unpack(flat, sizes)
    H = np.asarray(X, float)
    cache = [H]
    for li, (W, b) in enumerate(params):
        Z = H @ W.T + b
        if li < len(params) - 1:
            cache.append(Z)
            H = silu(Z)
            cache.append(H)
        else:
            H = Z
    return H, cache


def loss_and_grad(flat, X, T, sizes=SIZES):
    """Mean squared error over all outputs and its gradient (flat, same layout)."""
    params = unpack(flat, sizes)
    Y, cache = forward(flat, X, sizes)
    T = np.asarray(T, float)
    R = Y - T
    loss = np.mean(R * R)
    dZ = 2.0 * R / R.size
    grads = [None] * len(params)
    nl = len(params)
    for li in range(nl - 1, -1, -1):
        W, _ = params[li]
        Hin = cache[0] if li == 0 else cache[2 * li]
        grads[li] = (dZ.T @ Hin, dZ.sum(0))
        if li > 0:
            dH = dZ @ W
            dZ = dH * dsilu(cache[2 * li - 1])
    return loss, pack(grads)


def adam(flat, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (flat, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
