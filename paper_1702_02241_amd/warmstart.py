"""Learned warm start for streaming windows (driver around rpca_warm.h).

A window is `frames` consecutive columns of a column-major video matrix, so
with X stored as an (n_frames, m) device tensor a window is the contiguous
row slice ``X[t : t + frames]``.  Every step below runs in librpca kernels;
this module only orders the calls and holds the device buffers:

  * training pairs: solve a window from the randomized-SVD cold start
    (``rpca_solve``), pool its U* to the feature resolution
    (``rpca_pool_rows``) and keep (features, pool(U*), V*);
  * training: minibatch Adam on the rotation-invariant product loss
    (``rpca_mlp_train_step``);
  * prediction: features -> forward pass -> upsample U (``rpca_upsample_rows``)
    -> ``rpca_solve`` from the predicted factors, with the cold start as the
    fallback when the predicted start has the larger objective.

The feature normalisation (per-feature shift and scale) is fitted once on
the host from the training features; the kernels apply it.
"""
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import rpca as R
from . import synth
from . import torch_api as T


@dataclass
class WindowSpec:
    width: int = 320
    height: int = 240
    frames: int = 100       # window length (columns)
    stride: int = 10        # frames between consecutive windows
    factor: int = 4         # pooling factor of the features and of U_low
    k: int = 10
    lam_s: float = 0.05
    lam_l: float = None     # default 0.05 * sqrt(m)

    @property
    def m(self):
        return self.width * self.height

    @property
    def mu(self):
        return (self.width // self.factor) * (self.height // self.factor)

    @property
    def d_in(self):
        return 2 * self.mu + self.frames

    @property
    def lam(self):
        return self.lam_l if self.lam_l is not None else 0.05 * np.sqrt(self.m)


def video_tensor(spec, n_frames, seed, device):
    """Synthetic video (the seeded generator of synth.video_frames) as an
    (n_frames, m) float32 device tensor: row t is frame t."""
    X, _, _ = synth.video_frames(n_frames=n_frames, width=spec.width, height=spec.height, seed=seed)
    return torch.from_numpy(np.ascontiguousarray(X.T.astype(np.float32))).to(device)


def window_starts(n_frames, spec):
    return list(range(0, n_frames - spec.frames + 1, spec.stride))


class WarmStart:
    def __init__(self, spec, d_h=512, max_batch=64, seed=0, device="cuda"):
        self.spec = spec
        self.device = torch.device(device)
        self.net = T.WarmNet(spec.d_in, d_h, spec.mu, spec.frames, spec.k, max_batch=max_batch, seed=seed)
        self.ctx = T.Context(spec.m, spec.frames, spec.k, spec.lam_s, spec.lam)
        self.shift = None
        self.scale = None

    def close(self):
        self.net.close()
        self.ctx.close()

    # -- features ---------------------------------------------------------
    def features(self, Xw, normalised=True):
        s = self.spec
        if normalised and self.shift is not None:
            return T.window_features(Xw, s.width, s.height, s.frames, s.factor, self.shift, self.scale)
        return T.window_features(Xw, s.width, s.height, s.frames, s.factor)

    def fit_normaliser(self, raw):
        """raw: (N, d_in) device features.  Shift = mean, scale = 1/std (host statistics)."""
        a = raw.cpu().numpy().astype(np.float64)
        mu = a.mean(axis=0)
        sd = a.std(axis=0)
        sc = 1.0 / np.maximum(sd, 1e-3 * max(float(sd.max()), 1e-12))
        self.shift = torch.from_numpy(mu.astype(np.float32)).to(self.device)
        self.scale = torch.from_numpy(sc.astype(np.float32)).to(self.device)

    # -- solver -----------------------------------------------------------
    def solve(self, Xw, start=None, **opts):
        """Solve one window; start = (U, V) device tensors or None for the cold start."""
        s = self.spec
        if start is None:
            U = torch.empty(s.m, s.k, dtype=torch.float32, device=self.device)
            V = torch.empty(s.frames, s.k, dtype=torch.float32, device=self.device)
            init = R.RPCA_INIT_RSVD
        else:
            U, V = (t.clone() for t in start)
            init = R.RPCA_INIT_GIVEN
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = self.ctx.solve(Xw, U, V, init=init, **opts)
        torch.cuda.synchronize()
        return rc, info, U, V, time.perf_counter() - t0

    def objective(self, Xw, U, V):
        f, _, _ = self.ctx.objgrad(Xw, U, V)
        return float(f.item())

    # -- training data ----------------------------------------------------
    def build_dataset(self, videos, log=None):
        """videos: list of (n_frames, m) device tensors.  Solves every window
        from the cold start, fits the feature normalisation on the raw
        features, and returns normalised features, pooled U*, V* and the
        per-window solve records, in a seeded shuffled order."""
        s = self.spec
        raw, TUs, TVs, recs = [], [], [], []
        for vi, Xv in enumerate(videos):
            for t in window_starts(Xv.shape[0], s):
                Xw = Xv[t:t + s.frames]
                raw.append(self.features(Xw, normalised=False))
                rc, info, U, V, sec = self.solve(Xw)
                TUs.append(T.pool_rows(U, s.width, s.height, s.factor))
                TVs.append(V)
                recs.append((vi, t, rc, info.iters, info.certified, sec))
            if log:
                log(f"dataset: video {vi + 1}/{len(videos)}, {len(raw)} windows")
        self.fit_normaliser(torch.stack(raw))
        feats = [self.features(videos[vi][t:t + s.frames]) for vi, t, *_ in recs]
        perm = np.random.default_rng(12345).permutation(len(feats))
        F = torch.stack([feats[i] for i in perm])
        TU = torch.stack([TUs[i] for i in perm])
        TV = torch.stack([TVs[i] for i in perm])
        return F, TU, TV, [recs[i] for i in perm]

    # -- training ---------------------------------------------------------
    def train(self, F, TU, TV, epochs, batch=64, lr=1e-3, log=None):
        """Minibatch Adam over contiguous batches of the (shuffled) dataset."""
        N = F.shape[0]
        nb = max(1, N // batch)
        order = np.random.default_rng(7)
        losses = []
        for ep in range(epochs):
            acc = 0.0
            for b in order.permutation(nb):
                sl = slice(b * batch, (b + 1) * batch)
                loss = self.net.train_step(F[sl], TU[sl], TV[sl], lr)
                acc += float(loss.item())
            losses.append(acc / nb)
            if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
                log(f"epoch {ep}: loss {losses[-1]:.6g}")
        return losses

    def eval_loss(self, F, TU, TV, batch=64):
        N = F.shape[0]
        tot, cnt = 0.0, 0
        for b0 in range(0, N, batch):
            sl = slice(b0, min(N, b0 + batch))
            nb = sl.stop - sl.start
            loss = self.net.loss_grad(F[sl], TU[sl], TV[sl])
            tot += float(loss.item()) * nb
            cnt += nb
        return tot / cnt

    # -- prediction -------------------------------------------------------
    def predict(self, Xw):
        s = self.spec
        x = self.features(Xw).reshape(1, -1)
        y = self.net.forward(x).reshape(-1)
        U_low = y[: s.mu * s.k].reshape(s.mu, s.k)
        V = y[s.mu * s.k:].reshape(s.frames, s.k).clone()
        U = T.upsample_rows(U_low.contiguous(), s.width, s.height, s.factor)
        return U, V

    def start_for(self, Xw):
        """Predicted start, or the cold start when it has the larger objective.
        Returns ((U, V) or None, f_pred, f_cold)."""
        U, V = self.predict(Xw)
        f_pred = self.objective(Xw, U, V)
        Uc, Vc = self.ctx.init_rsvd(Xw)
        f_cold = self.objective(Xw, Uc, Vc)
        return ((U, V) if f_pred < f_cold else None), f_pred, f_cold


def low_rank_distance(U, V, Ur, Vr):
    """||U V^T - Ur Vr^T||_F / ||Ur Vr^T||_F through k x k traces (FP64 on the host)."""
    U, V, Ur, Vr = (np.asarray(a.cpu().numpy() if hasattr(a, "cpu") else a, np.float64) for a in (U, V, Ur, Vr))
    a = np.sum((U.T @ U) * (V.T @ V))
    b = np.sum((U.T @ Ur) * (V.T @ Vr))
    c = np.sum((Ur.T @ Ur) * (Vr.T @ Vr))
    return float(np.sqrt(max(a - 2 * b + c, 0.0) / c))


def shift_start(U_prev, V_prev, Xw, spec):
    """The trivial warm start for a window that follows the previous one by
    ``spec.stride`` frames: the previous U, the previous V moved up by stride rows,
    and for the stride new frames the ridge fit x ~ U v, v = (U^T U + lam_L I)^-1 U^T x
    (a baseline for the learned start; its small k x k algebra runs on the host)."""
    s = spec
    U = U_prev.detach().cpu().numpy().astype(np.float64)
    Xn = Xw[s.frames - s.stride:].detach().cpu().numpy().astype(np.float64)  # stride x m
    G = U.T @ U + s.lam * np.eye(s.k)
    Vn = np.linalg.solve(G, U.T @ Xn.T).T
    V = np.vstack([V_prev.detach().cpu().numpy().astype(np.float64)[s.stride:], Vn])
    return U_prev.clone(), torch.from_numpy(V.astype(np.float32)).to(U_prev.device)


def evaluate_stream(ws, Xv, starts, keep=(), log=None):
    """Solve the windows of one video from three starts and record, per window and
    start, the accepted iterations, the time to a certified solution (the start's
    construction included) and the certificate's verdict:

      cold     -- the randomized-SVD start inside rpca_solve;
      trivial  -- ``shift_start`` from this chain's previous certified window;
      learned  -- the network's prediction, used as it is;
      rule     -- the prediction or the cold start, whichever has the lower objective.

    ``keep``: window starts whose solutions (U, V per start) are returned for an
    outside comparison."""
    s = ws.spec
    recs, kept = [], {}
    prev = None
    for wi, t in enumerate(starts):
        Xw = Xv[t:t + s.frames]
        rec = {"t": int(t)}
        sol = {}
        rc, info, U, V, sec = ws.solve(Xw)
        rec["cold"] = (info.iters, 1e3 * sec, int(info.certified), info.f)
        sol["cold"] = (U, V)
        if prev is not None and t - prev[0] == s.stride:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = shift_start(prev[1], prev[2], Xw, s)
            build = time.perf_counter() - t0
            rc, info, U2, V2, sec = ws.solve(Xw, st)
            rec["trivial"] = (info.iters, 1e3 * (build + sec), int(info.certified), info.f)
            sol["trivial"] = (U2, V2)
            prev = (t, U2, V2)
        else:
            prev = (t, U, V)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Up, Vp = ws.predict(Xw)
        torch.cuda.synchronize()
        build = time.perf_counter() - t0
        rc, info, U3, V3, sec = ws.solve(Xw, (Up, Vp))
        rec["learned"] = (info.iters, 1e3 * (build + sec), int(info.certified), info.f)
        sol["learned"] = (U3, V3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start, f_pred, f_cold = ws.start_for(Xw)
        torch.cuda.synchronize()
        build = time.perf_counter() - t0
        rc, info, U4, V4, sec = ws.solve(Xw, start)
        rec["rule"] = (info.iters, 1e3 * (build + sec), int(info.certified), info.f,
                       "learned" if start is not None else "cold")
        recs.append(rec)
        if t in keep:
            kept[int(t)] = {k: (a.detach().cpu().numpy(), b.detach().cpu().numpy()) for k, (a, b) in sol.items()}
        if log and (wi % 50 == 0 or wi == len(starts) - 1):
            log(f"stream: window {wi + 1}/{len(starts)} (frame {t}): " + ", ".join(
                f"{k} {rec[k][0]} it {rec[k][1]:.1f} ms" for k in ("cold", "trivial", "learned", "rule") if k in rec))
    return recs, kept
