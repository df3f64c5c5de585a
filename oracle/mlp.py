"""Learned CG preconditioner network — TEST INFRASTRUCTURE ONLY (see the
package docstring).

The paper solves each local first-order equation with conjugate gradients
(the local linear equation of the two-site step, Eq. pt2 restricted to the
window).  The learned preconditioner replaces the Jacobi preconditioner
D^-1 by s_B D^-1 on every block B of the two-site tensor, with one positive
scale per block predicted by a small network from statistics of the
diagonal; a preconditioner that stays symmetric positive definite leaves
the converged solution unchanged, so only the iteration count depends on
it.  The paper does not describe such a network: this module fixes the
arithmetic the GPU kernels must reproduce, in float64.

Network (F = 8 inputs, two tanh layers of 64, softplus output):
  a1 = W1 x + b1, h1 = tanh(a1); a2 = W2 h1 + b2, h2 = tanh(a2);
  o = w3 . h2 + b3;  s = softplus(o) = log(1 + e^o).
Loss over n samples with targets t > 0:  L = (1/n) sum (log s - log t)^2.
Flat parameter layout (N_PARAMS = 4801): W1[64][8] row major, b1[64],
W2[64][64] row major, b2[64], w3[64], b3.
Adam: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments.

CG starts from the previous window's state x0, so the preconditioner's job is
to map the initial residual r0 = -b - A x0 onto the initial error
e0 = x - x0 (A e0 = r0).  Features of a block B with diagonal values d
(all > 0), initial residual r0 and the window's whole initial residual r_all,
window i of n - 1:
  mean log d, std log d, min log d - mean, max log d - mean, log rows,
  log cols, log(|r0_B| / |r_all|) (norms floored at 1e-300), i / (n - 2).
Target of B from the converged solution: with z = r0 / d (the Jacobi step),
t = <e0_B, z_B> / <z_B, z_B>, the scale that best fits e0_B by z_B.
"""
import numpy as np

F, H = 8, 64
N_PARAMS = H * F + H + H * H + H + H + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def softplus(o):
    return np.maximum(o, 0.0) + np.log1p(np.exp(-np.abs(o)))


def forward(p, X):
    """Scales s (n,) for feature rows X (n, F)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return softplus(h2 @ w3 + b3)


def loss(p, X, t):
    s = forward(p, X)
    return float(np.mean((np.log(s) - np.log(t)) ** 2))


def loss_and_grad(p, X, t):
    """Loss and its gradient with respect to the flat parameters (backpropagation)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    o = h2 @ w3 + b3
    s = softplus(o)
    r = np.log(s) - np.log(t)
    L = float(np.mean(r ** 2))
    sig = 1.0 / (1.0 + np.exp(-o))
    do = (2.0 / n) * r * sig / s                  # dL/do per sample
    dw3 = h2.T @ do
    db3 = do.sum()
    da2 = np.outer(do, w3) * (1.0 - h2 ** 2)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * (1.0 - h1 ** 2)
    dW1 = da1.T @ X
    db1 = da1.sum(axis=0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])
    return L, g


def adam_step(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def block_features(d, r0, r_all_norm, window, n_sites):
    """Features of one block (d, r0: the block's diagonal and initial residual, 2-D)."""
    ld = np.log(d.ravel())
    mu = ld.mean()
    rn = max(np.linalg.norm(r0), 1e-300)
    return np.array([mu, ld.std(), ld.min() - mu, ld.max() - mu, np.log(d.shape[0]), np.log(d.shape[1]),
                     np.log(rn / max(r_all_norm, 1e-300)), window / (n_sites - 2)])


def block_target(d, r0, e0):
    z = r0 / d
    zz = float(np.sum(z * z))
    return float(np.sum(e0 * z)) / zz if zz > 0 else None
