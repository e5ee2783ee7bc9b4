"""Pins for oracle.mlp: hand-written backward against central finite differences,
Adam against its defining recursion, pooling/upsampling round trips."""
import numpy as np

from oracle import mlp


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    B, din, dh, mu, nv, k = 3, 7, 6, 5, 4, 2
    dout = mu * k + nv * k
    x = rng.normal(size=(B, din))
    W1, b1 = rng.normal(size=(din, dh)) * 0.5, rng.normal(size=dh) * 0.1
    W2, b2 = rng.normal(size=(dh, dout)) * 0.5, rng.normal(size=dout) * 0.1
    T = rng.normal(size=(B, mu, nv))
    loss, dW1, db1, dW2, db2 = mlp.loss_grad(x, T, W1, b1, W2, b2, mu, nv, k)
    h = 1e-6
    for P, dP in ((W1, dW1), (b1, db1), (W2, dW2), (b2, db2)):
        flat = P.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 13)):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss_grad(x, T, W1, b1, W2, b2, mu, nv, k)[0]
            flat[idx] = old - h
            lm = mlp.loss_grad(x, T, W1, b1, W2, b2, mu, nv, k)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - dP.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_adam_first_step_is_signed_lr():
    # with bias correction the first Adam step is -lr * g/(|g| + eps) elementwise
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_pool_and_upsample_are_consistent():
    rng = np.random.default_rng(1)
    A = rng.normal(size=(12 * 8, 3))
    low = mlp.downsample_rows(A, 12, 8, 4)
    assert low.shape == (6, 3)
    up = mlp.upsample_rows(low, 12, 8, 4)
    assert np.allclose(mlp.downsample_rows(up, 12, 8, 4), low)
    assert abs(A[:4].mean() - 0) < 10  # shape sanity
    # first low-res pixel is the mean of the top-left 4x4 block
    blk = A.reshape(8, 12, 3)[:4, :4].mean(axis=(0, 1))
    assert np.allclose(low[0], blk)
