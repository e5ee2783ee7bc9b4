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


def test_adam_constant_gradient_closed_form_at_steps_2_and_3():
    # For a constant gradient g, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    # bias-corrected moments are exactly g and g^2 and every step moves by
    # -lr * g / (|g| + eps): the closed form of Kingma & Ba's correction.
    g = np.array([0.7, -1.5, 4e-3])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    b1, b2, lr, eps = 0.9, 0.999, 0.05, 1e-8
    for t in (1, 2, 3):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        assert np.allclose(m, (1 - b1 ** t) * g, rtol=1e-13)
        assert np.allclose(v, (1 - b2 ** t) * g * g, rtol=1e-13)
        assert np.allclose(p, -t * lr * g / (np.abs(g) + eps), rtol=1e-12)


def test_adam_varying_gradients_match_weighted_sums():
    # Unrolled moments: m_t = (1 - b1) sum_s b1^(t-s) g_s, v_t = (1 - b2) sum_s b2^(t-s) g_s^2.
    # Hand-checked two-step value for one coordinate (b1 = 0.5, b2 = 0.75, lr = 1, eps = 0):
    # g1 = 2, g2 = -1: m2 = 0.25*2 + 0.5*(-1) = 0, so the second step does not move p.
    p, m, v = mlp.adam_step(np.array([0.0]), np.array([2.0]), np.zeros(1), np.zeros(1), 1,
                            lr=1.0, beta1=0.5, beta2=0.75, eps=0.0)
    assert np.allclose(p, [-1.0])
    p2, m2, v2 = mlp.adam_step(p, np.array([-1.0]), m, v, 2, lr=1.0, beta1=0.5, beta2=0.75, eps=0.0)
    assert m2[0] == 0.0 and np.allclose(p2, p)
    assert np.isclose(v2[0], 0.25 * (0.75 * 4.0 + 1.0))
    rng = np.random.default_rng(3)
    gs = rng.normal(size=(3, 5))
    b1, b2, lr, eps = 0.8, 0.95, 0.01, 1e-8
    p, m, v = np.zeros(5), np.zeros(5), np.zeros(5)
    for t in (1, 2, 3):
        p_prev = p
        p, m, v = mlp.adam_step(p, gs[t - 1], m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        ms = (1 - b1) * sum(b1 ** (t - s) * gs[s - 1] for s in range(1, t + 1))
        vs = (1 - b2) * sum(b2 ** (t - s) * gs[s - 1] ** 2 for s in range(1, t + 1))
        assert np.allclose(m, ms, rtol=1e-13) and np.allclose(v, vs, rtol=1e-13)
        step = lr * (ms / (1 - b1 ** t)) / (np.sqrt(vs / (1 - b2 ** t)) + eps)
        assert np.allclose(p, p_prev - step, rtol=1e-12, atol=1e-15)


def test_window_features_hand_computed():
    # 4 x 2 pixel frames (pixel i = y * width + x), pooled 2 x 2, two frames.
    # Frame 0 holds 1..8, frame 1 twice that.  Low-res block (0, 0) covers pixels
    # 0, 1, 4, 5 and block (0, 1) pixels 2, 3, 6, 7: frame means 3.5, 5.5 and 7, 11.
    # Temporal mean 5.25, 8.25; population std |a - b| / 2 = 1.75, 2.75;
    # per-frame means 4.5 and 9.
    f0 = np.arange(1.0, 9.0)
    Xw = np.stack([f0, 2.0 * f0], axis=1)  # 8 pixels x 2 frames
    feat = mlp.window_features(Xw, width=4, height=2, factor=2)
    assert np.allclose(feat, [5.25, 8.25, 1.75, 2.75, 4.5, 9.0], rtol=0, atol=1e-15)


def test_window_features_by_loops():
    # the same statistics by explicit loops over blocks, frames and pixels
    rng = np.random.default_rng(5)
    W, H, fct, n = 6, 4, 2, 5
    Xw = rng.uniform(size=(W * H, n))
    feat = mlp.window_features(Xw, W, H, fct)
    nb = (W // fct) * (H // fct)
    low = np.zeros((n, nb))
    for t in range(n):
        for by in range(H // fct):
            for bx in range(W // fct):
                acc = 0.0
                for dy in range(fct):
                    for dx in range(fct):
                        acc += Xw[(by * fct + dy) * W + bx * fct + dx, t]
                low[t, by * (W // fct) + bx] = acc / (fct * fct)
    mean = [sum(low[t, b] for t in range(n)) / n for b in range(nb)]
    std = [np.sqrt(sum((low[t, b] - mean[b]) ** 2 for t in range(n)) / n) for b in range(nb)]
    fmean = [sum(Xw[i, t] for i in range(W * H)) / (W * H) for t in range(n)]
    assert np.allclose(feat, np.concatenate([mean, std, fmean]), rtol=1e-13, atol=1e-15)
