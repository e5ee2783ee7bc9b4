"""Two-layer MLP for warm-starting factors, FP64 (oracle; tests only).

The paper has no learned component: its initialisation is a randomized SVD
(Sec. 4.2).  The warm-start network proposes factors for a window of a
streaming video from cheap window statistics; its target is the converged
low-resolution low-rank part, compared through the rotation-invariant product
U_hat V_hat^T (Theorem 1: factors are unique only up to an orthogonal Q).

Layout (shared only as a convention with the GPU kernels, not as code):
    x  : B x d_in            row-major features
    W1 : d_in x d_h,  b1 : d_h
    W2 : d_h x d_out, b2 : d_out,  d_out = mu*k + nv*k
    y  = relu(x W1 + b1) W2 + b2;  y[:, :mu*k] is U_hat (mu x k, row-major),
                                   y[:, mu*k:] is V_hat (nv x k, row-major)
    loss = (1/B) sum_b ||U_hat_b V_hat_b^T - T_b||_F^2

Backward is written out by hand.  Adam follows Kingma & Ba with bias
correction.  Window statistics use the population standard deviation
(divide by the frame count).  Pins (tests/test_oracle_mlp.py): central finite
differences of ``loss`` in FP64; Adam against the closed form for a constant
gradient at steps 1-3 and against the unrolled moment sums for varying
gradients, with a two-step case worked by hand; the window statistics against
a 4 x 2 pixel, two-frame case worked by hand and against explicit loops.
"""
import numpy as np


def forward(x, W1, b1, W2, b2):
    z1 = x @ W1 + b1
    h = np.maximum(z1, 0.0)
    y = h @ W2 + b2
    return z1, h, y


def split(y, mu, nv, k):
    B = y.shape[0]
    return y[:, : mu * k].reshape(B, mu, k), y[:, mu * k:].reshape(B, nv, k)


def loss_grad(x, T, W1, b1, W2, b2, mu, nv, k):
    """Return (loss, dW1, db1, dW2, db2) for targets T (B x mu x nv)."""
    B = x.shape[0]
    z1, h, y = forward(x, W1, b1, W2, b2)
    Uh, Vh = split(y, mu, nv, k)
    Rz = np.einsum("bik,bjk->bij", Uh, Vh) - T
    loss = float(np.sum(Rz * Rz)) / B
    dUh = (2.0 / B) * np.einsum("bij,bjk->bik", Rz, Vh)
    dVh = (2.0 / B) * np.einsum("bij,bik->bjk", Rz, Uh)
    dy = np.concatenate([dUh.reshape(B, -1), dVh.reshape(B, -1)], axis=1)
    dW2 = h.T @ dy
    db2 = dy.sum(axis=0)
    dh = dy @ W2.T
    dz1 = dh * (z1 > 0)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    return loss, dW1, db1, dW2, db2


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t is the 1-based step count).  Returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def window_features(Xw, width, height, factor):
    """Window statistics: per-block temporal mean and std of the frames
    downsampled by ``factor`` in each direction, and the per-frame means."""
    n = Xw.shape[1]
    fr = Xw.T.reshape(n, height // factor, factor, width // factor, factor)
    low = fr.mean(axis=(2, 4)).reshape(n, -1)          # n x (h/f * w/f)
    return np.concatenate([low.mean(axis=0), low.std(axis=0), Xw.mean(axis=0)])


def downsample_rows(A, width, height, factor):
    """Average-pool the pixel rows of an (height*width) x c matrix."""
    c = A.shape[1]
    t = A.reshape(height // factor, factor, width // factor, factor, c)
    return t.mean(axis=(1, 3)).reshape(-1, c)


def upsample_rows(A, width, height, factor):
    """Nearest-neighbour upsampling of a low-resolution (h/f * w/f) x c matrix."""
    c = A.shape[1]
    t = A.reshape(height // factor, width // factor, c)
    t = np.repeat(np.repeat(t, factor, axis=0), factor, axis=1)
    return t.reshape(-1, c)
