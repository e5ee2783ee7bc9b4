"""Frank-Wolfe with the sparse part marginalised (Sec. 6.2, Alg. 1), FP64
(oracle; test infrastructure only).

Problem (the program of Sec. 6.2, equivalent to SPCP): over (L, t) with
||L||_* <= t, minimise  lam_l t + phi(L),  phi the Huber marginal of
oracle.objective.  Each iteration of Alg. 1, as read here (the printed
algorithm is garbled in two places; the readings follow the Frank-Wolfe scheme
with a nuclear-norm bound variable that it extends):

  1. G_k = grad phi(L_k) = P_Omega(L_k + S_k - X) with S_k = shrink(X - L_k).
  2. Linear minimisation over the unit nuclear ball: Y_k = -u v^T with (sigma,
     u, v) the top singular triplet of G_k, so <G_k, Y_k> = -sigma.
  3. The bound variable lies in [0, B_k]: if lam_l >= sigma the vertex is
     (V_k, Vt_k) = (0, 0), else (B_k Y_k, B_k).
  4. Step size: exact minimiser over [0, 1] of the quadratic model
     1/2 ||G_k + eta P_Omega(V_k - L_k)||^2 + lam_l ((1 - eta) t_k + eta Vt_k),
     i.e. the printed line search with S_k held fixed (reading: its last term is
     eta lam_l Vt_k; the printed eta lam_l t_k would make t's step free).  The
     model majorises the marginal objective and equals it at eta = 0, so the
     objective never increases.
  5. L_{k+1} = (1 - eta) L_k + eta V_k,  t_{k+1} = (1 - eta) t_k + eta Vt_k.
  6. B_{k+1} = (phi(L_{k+1}) + lam_l t_{k+1}) / lam_l (reading: the printed
     bound reuses the start's residual; any objective value over lam_l bounds
     ||L*||_*, and the current one is the tightest at hand).  B_0 = phi(0)/lam_l.

The Frank-Wolfe gap <G_k, L_k - V_k> + lam_l (t_k - Vt_k) bounds the
objective's distance to the optimum (convexity; the optimum is feasible for
t <= B_k).

Pins (tests/test_oracle_frank_wolfe.py): the step size against a brute-force
minimisation of the model; the gap bounds F_k - F* with F* from FISTA-SVT
(oracle.convex, an independent solver); monotone objective; feasibility
||L_k||_* <= t_k; convergence to the lam_s -> infinity closed form
(singular-value soft threshold of X).
"""
import numpy as np

from .objective import grad_phi, phi


def _omega(mask, shape):
    if mask is None:
        return np.ones(shape, dtype=np.float64)
    return (np.asarray(mask) != 0).astype(np.float64)


def top_triplet(G):
    """(sigma, u, v): top singular triplet of G (LAPACK SVD)."""
    Us, s, Vt = np.linalg.svd(G, full_matrices=False)
    return float(s[0]), Us[:, 0], Vt[0]


def step_size(G, L, t, V, Vt, lam_l, mask=None):
    """Minimiser over [0, 1] of 1/2||G + eta P_Omega(V - L)||^2 + lam_l((1-eta) t + eta Vt)."""
    W = _omega(mask, G.shape)
    D = W * (V - L)
    dd = float(np.sum(D * D))
    if dd <= 0.0:
        return 0.0
    eta = -(float(np.sum(G * D)) + lam_l * (Vt - t)) / dd
    return min(max(eta, 0.0), 1.0)


def fw_iteration(L, t, X, lam_s, lam_l, mask=None):
    """One iteration of Alg. 1 from (L_k, t_k).  Returns (L_{k+1}, t_{k+1}, info)
    with info = dict(F, gap, sigma, eta, B, step) describing iterate k."""
    L = np.asarray(L, np.float64)
    G = grad_phi(L, X, lam_s, mask)
    phiL = phi(L, X, lam_s, mask)
    B = phiL / lam_l + t
    sigma, u, v = top_triplet(G)
    if lam_l >= sigma:
        V, Vt = np.zeros_like(L), 0.0
    else:
        V, Vt = -B * np.outer(u, v), B
    gap = float(np.sum(G * (L - V))) + lam_l * (t - Vt)
    eta = step_size(G, L, t, V, Vt, lam_l, mask)
    Ln = (1.0 - eta) * L + eta * V
    tn = (1.0 - eta) * t + eta * Vt
    return Ln, tn, dict(F=phiL + lam_l * t, gap=gap, sigma=sigma, eta=eta, B=B,
                        step=bool(Vt > 0))


def fw_solve(X, lam_s, lam_l, mask=None, max_iter=1000, tol=1e-6, L0=None, t0=0.0):
    """Alg. 1 from (L0, t0) (default 0, 0) until gap <= tol * F or max_iter.
    Returns dict(L, t, F, gap, iters, hist) with hist a list of per-iterate info."""
    X = np.asarray(X, np.float64)
    L = np.zeros_like(X) if L0 is None else np.array(L0, np.float64)
    t = float(t0)
    hist = []
    for it in range(max_iter + 1):
        Ln, tn, info = fw_iteration(L, t, X, lam_s, lam_l, mask)
        hist.append(info)
        if info["gap"] <= tol * max(info["F"], 1e-300) or it == max_iter:
            break
        L, t = Ln, tn
    last = hist[-1]
    return dict(L=L, t=t, F=last["F"], gap=last["gap"], iters=len(hist) - 1, hist=hist)
