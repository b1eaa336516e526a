"""CPU oracle of the learned reliability refinement (test infrastructure only).

The refinement network is not part of the paper; it is this project's addition that re-ranks
BP's soft output before LSD consumes it (LSD only uses the order of its input LLRs, Sec. 4.1
step 2).  The definition below is the one the HIP kernels implement; here it is written out in
float64 numpy, one shot at a time, with its gradient derived by hand (checked against finite
differences in the tests).

Per shot, with H (m x n), BP posteriors L, prior LLRs lam, syndrome s, sigma_i = 1 - 2 s_i:

    x_j      = (tanh(L_j / 8), lam_j / 8)
    h0_j     = relu(W0 x_j + b0)                                   (32)
    for l = 1..3:
      m_i    = (1/deg_i) sum_{j in N(i)} h_{l-1,j}
      c_i    = relu(A_l m_i + sigma_i a_l)                         (32)
      g_j    = (1/deg_j) sum_{i in N(j)} c_i
      h_l,j  = relu(B_l h_{l-1,j} + C_l g_j + b_l)                 (32)
    Delta_j  = w . h_3,j + b_out
    L'_j     = L_j + Delta_j
    loss     = mean_j [ softplus(-L'_j) + e_j L'_j ]               (BCE of P(e_j=1) = sigmoid(-L'_j))

Parameters are one flat float vector in the order of PARAM_LAYOUT.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expit

HID = 32
LAYERS = 3
PARAM_LAYOUT = ([("W0", (HID, 2)), ("b0", (HID,))] +
                [(f"{nm}{l}", shp) for l in range(1, LAYERS + 1)
                 for nm, shp in (("A", (HID, HID)), ("a", (HID,)), ("B", (HID, HID)),
                                 ("C", (HID, HID)), ("b", (HID,)))] +
                [("w", (HID,)), ("bo", (1,))])
N_PARAMS = int(sum(int(np.prod(s)) for _, s in PARAM_LAYOUT))


def unpack(theta: np.ndarray) -> dict:
    out, off = {}, 0
    for name, shp in PARAM_LAYOUT:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[off:off + k], dtype=np.float64).reshape(shp)
        off += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in PARAM_LAYOUT])


def init_params(seed: int = 0, zero_output: bool = True) -> np.ndarray:
    """Glorot-style uniform init; the output layer starts at zero so Delta == 0 initially."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in PARAM_LAYOUT:
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            p[name] = rng.uniform(-lim, lim, size=shp)
        else:
            p[name] = np.zeros(shp)
    if not zero_output:
        p["w"] = rng.uniform(-0.3, 0.3, size=(HID,))
    return pack(p)


def _graph(H):
    H = np.asarray(H, dtype=np.float64)
    deg_c = H.sum(1)
    deg_f = H.sum(0)
    return H, deg_c, deg_f


def forward(theta, H, L, lam, s, keep=False):
    """One shot -> Delta (n,) [and the activations when keep]."""
    p = unpack(theta)
    H, deg_c, deg_f = _graph(H)
    sigma = 1.0 - 2.0 * (np.asarray(s) & 1)
    x = np.stack([np.tanh(np.asarray(L, np.float64) / 8.0), np.asarray(lam, np.float64) / 8.0], axis=1)
    u0 = x @ p["W0"].T + p["b0"]
    h = np.maximum(u0, 0.0)
    acts = {"x": x, "u0": u0, "h0": h}
    for l in range(1, LAYERS + 1):
        m = (H @ h) / deg_c[:, None]
        v = m @ p[f"A{l}"].T + sigma[:, None] * p[f"a{l}"]
        c = np.maximum(v, 0.0)
        g = (H.T @ c) / deg_f[:, None]
        u = h @ p[f"B{l}"].T + g @ p[f"C{l}"].T + p[f"b{l}"]
        acts[f"m{l}"], acts[f"v{l}"], acts[f"c{l}"], acts[f"g{l}"], acts[f"u{l}"] = m, v, c, g, u
        h = np.maximum(u, 0.0)
        acts[f"h{l}"] = h
    delta = h @ p["w"] + p["bo"][0]
    return (delta, acts) if keep else delta


def loss_and_grad(theta, H, L, lam, s, e):
    """Mean BCE over the shot's faults and its gradient w.r.t. theta (hand-derived)."""
    p = unpack(theta)
    Hm, deg_c, deg_f = _graph(H)
    n = Hm.shape[1]
    delta, A = forward(theta, H, L, lam, s, keep=True)
    Lp = np.asarray(L, np.float64) + delta
    e = np.asarray(e, np.float64)
    loss = float(np.mean(np.logaddexp(0.0, -Lp) + e * Lp))
    # d loss / d L'_j = (e_j - sigmoid(-L'_j)) / n ; L' = L + Delta
    dD = (e - expit(-Lp)) / n
    sigma = 1.0 - 2.0 * (np.asarray(s) & 1)
    g = {k: np.zeros_like(v) for k, v in p.items()}
    g["w"] = A[f"h{LAYERS}"].T @ dD
    g["bo"] = np.array([dD.sum()])
    dh = np.outer(dD, p["w"])
    for l in range(LAYERS, 0, -1):
        du = dh * (A[f"u{l}"] > 0)
        h_prev = A[f"h{l - 1}"]
        g[f"B{l}"] = du.T @ h_prev
        g[f"C{l}"] = du.T @ A[f"g{l}"]
        g[f"b{l}"] = du.sum(0)
        dh = du @ p[f"B{l}"]
        dgv = du @ p[f"C{l}"]
        dc = (Hm @ (dgv / deg_f[:, None]))
        dv = dc * (A[f"v{l}"] > 0)
        g[f"A{l}"] = dv.T @ A[f"m{l}"]
        g[f"a{l}"] = (sigma[:, None] * dv).sum(0)
        dm = dv @ p[f"A{l}"]
        dh = dh + Hm.T @ (dm / deg_c[:, None])
    du0 = dh * (A["u0"] > 0)
    g["W0"] = du0.T @ A["x"]
    g["b0"] = du0.sum(0)
    return loss, pack(g)


def batch_loss_and_grad(theta, H, Ls, lam, S, E):
    """Mean over shots of loss_and_grad."""
    tot, gt = 0.0, np.zeros(N_PARAMS)
    for b in range(len(Ls)):
        l, g = loss_and_grad(theta, H, Ls[b], lam, S[b], E[b])
        tot += l
        gt += g
    return tot / len(Ls), gt / len(Ls)
