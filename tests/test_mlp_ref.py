"""Pins of the float64 network reference (oracle/mlp_ref.py), CPU only."""
import numpy as np

from oracle import mlp_ref as M


def _case(seed, n=24):
    rng = np.random.default_rng(seed)
    w = M.init_params(rng)
    w[M.O_B1:M.O_W2] = rng.normal(0, 0.3, 64)
    w[M.O_B2:M.O_W3] = rng.normal(0, 0.3, 64)
    w[M.O_B3] = 0.2
    x = rng.normal(0, 1.0, (n, 8))
    y = (rng.random(n) < 0.3).astype(np.float64)
    return w, x, y


def test_gradient_equals_central_differences():
    """Every one of the 4801 partial derivatives, float64, roundings off."""
    for seed, pw in ((1, 1.0), (2, 7.5)):
        w, x, y = _case(seed)
        _, g = M.loss_and_grad(w, x, y, pw, round_act=False)
        h = 1e-6
        fd = np.zeros_like(w)
        for p in range(M.N_PARAM):
            wp = w.copy(); wp[p] += h
            wm = w.copy(); wm[p] -= h
            fd[p] = (M.loss_and_grad(wp, x, y, pw, False)[0] - M.loss_and_grad(wm, x, y, pw, False)[0]) / (2 * h)
        err = np.abs(fd - g)
        assert err.max() <= 1e-7 + 1e-5 * np.abs(g).max(), err.max()
        # no block of parameters is left without gradient
        for a, b in ((0, 512), (512, 576), (576, 4672), (4672, 4736), (4736, 4800), (4800, 4801)):
            assert np.abs(g[a:b]).max() > 0


def test_loss_at_zero_logit():
    """All-zero parameters give z = 0 and loss = mean(y pw + (1 - y)) log 2."""
    _, x, y = _case(3)
    for pw in (1.0, 4.0):
        loss, g = M.loss_and_grad(np.zeros(M.N_PARAM), x, y, pw)
        assert abs(loss - np.mean(y * pw + (1 - y)) * np.log(2.0)) < 1e-12
        # only b3 moves: dL/db3 = mean(pw y (1/2 - 1) + (1 - y) / 2)
        assert abs(g[M.O_B3] - np.mean(-0.5 * pw * y + 0.5 * (1 - y))) < 1e-12
        assert np.count_nonzero(g[:M.O_B3]) == 0


def test_forward_by_hand():
    """One sample through a network with a single active path."""
    w = np.zeros(M.N_PARAM)
    w[M.O_W1 + 3 * 8 + 2] = 2.0        # a1[3] = 2 x[2]
    w[M.O_W2 + 5 * 64 + 3] = -1.5      # a2[5] = -1.5 h1[3] + 1
    w[M.O_B2 + 5] = 1.0
    w[M.O_W3 + 5] = 4.0                # z = 4 h2[5] - 0.25
    w[M.O_B3] = -0.25
    x = np.zeros((2, 8)); x[0, 2] = 0.25; x[1, 2] = -1.0
    z, _ = M.forward(w, x, round_act=False)
    assert np.allclose(z, [4.0 * (1.0 - 1.5 * 0.5) - 0.25, 4.0 * 1.0 - 0.25])


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.140625, 1e-40])
    r = M.bf16_round(vals)
    # ties to even at 1 + 2^-8 (halfway between 1 and 1 + 2^-7)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == 1.0
    assert r[4] == -2.5 and r[5] == 3.140625
    assert np.array_equal(M.bits_to_float(M.bf16_bits(vals)), r)


def test_adam_first_step_closed_form():
    """First step: m-hat = g and v-hat = g^2, so the update is lr g/(|g|+eps)."""
    rng = np.random.default_rng(4)
    w = rng.normal(size=M.N_PARAM)
    g = rng.normal(size=M.N_PARAM)
    nw, m1, m2 = M.adam_step(w, np.zeros_like(w), np.zeros_like(w), g, 1, 0.01)
    assert np.allclose(nw, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)
