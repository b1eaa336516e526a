"""Pins for the float64 oracle of the learned refinement: the hand-derived gradient against
central finite differences, and the identity at zero output weights."""
import numpy as np

import oracle.learned as ol
from paper_2406_18655_amd.workloads import surface_hgp


def _shot(rng, code):
    L = rng.normal(size=code.n) * 4.0
    s = (rng.random(code.m) < 0.3).astype(np.uint8)
    e = (rng.random(code.n) < 0.2).astype(np.uint8)
    lam = np.full(code.n, np.log(19.0))
    return L, lam, s, e


def test_gradient_matches_finite_differences():
    code = surface_hgp(5)
    rng = np.random.default_rng(0)
    theta = ol.init_params(seed=3, zero_output=False)
    theta += rng.normal(size=theta.shape) * 0.05  # non-zero biases, away from ReLU kinks at 0
    shots = [_shot(rng, code) for _ in range(3)]
    Ls = [s[0] for s in shots]
    S = [s[2] for s in shots]
    E = [s[3] for s in shots]
    lam = shots[0][1]
    loss, g = ol.batch_loss_and_grad(theta, code.H, Ls, lam, S, E)
    idx = np.concatenate([rng.choice(ol.N_PARAMS, size=300, replace=False), [ol.N_PARAMS - 1, 0, 64]])
    eps = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (ol.batch_loss_and_grad(tp, code.H, Ls, lam, S, E)[0] -
              ol.batch_loss_and_grad(tm, code.H, Ls, lam, S, E)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-8, (k, fd, g[k])


def test_zero_output_is_identity():
    code = surface_hgp(5)
    rng = np.random.default_rng(1)
    theta = ol.init_params(seed=1, zero_output=True)
    L, lam, s, e = _shot(rng, code)
    assert np.array_equal(ol.forward(theta, code.H, L, lam, s), np.zeros(code.n))


def test_param_count_and_layout():
    assert ol.N_PARAMS == 9537
    p = ol.unpack(np.arange(ol.N_PARAMS, dtype=np.float64))
    assert p["W0"][0, 0] == 0 and p["A1"][0, 0] == 96 and p["bo"][0] == ol.N_PARAMS - 1


def test_forward_hand_computed_example():
    """Hand-worked forward pass on the length-3 repetition code (checks {0,1} and {1,2}) with
    weights that route one feature: h0 = relu(tanh(L/8)) in feature 0; layer 1 has A = B = C = I,
    a = -0.1 on feature 0 (syndrome sign enters as -1 for a flipped check); layers 2-3 pass h
    through (B = I, A = C = 0); the output reads feature 0.  With tanh(L/8) = (0.5, 0.25, 0.75)
    and s = (1, 0):
        m = (0.375, 0.5)             (check means of h0)
        c = (0.375 + 0.1, 0.5 - 0.1) = (0.475, 0.4)
        g = (0.475, (0.475 + 0.4)/2, 0.4) = (0.475, 0.4375, 0.4)
        h1 = h0 + g = (0.975, 0.6875, 1.15)  = Delta."""
    H = np.array([[1, 1, 0], [0, 1, 1]], dtype=np.uint8)
    p = {name: np.zeros(shp) for name, shp in ol.PARAM_LAYOUT}
    p["W0"][0, 0] = 1.0
    eye = np.eye(ol.HID)
    p["A1"], p["B1"], p["C1"] = eye, eye, eye
    p["a1"][0] = -0.1
    p["B2"], p["B3"] = eye, eye
    p["w"][0] = 1.0
    L = 8.0 * np.arctanh(np.array([0.5, 0.25, 0.75]))
    delta = ol.forward(ol.pack(p), H, L, np.full(3, 3.0), np.array([1, 0], dtype=np.uint8))
    np.testing.assert_allclose(delta, [0.975, 0.6875, 1.15], rtol=0, atol=1e-12)
