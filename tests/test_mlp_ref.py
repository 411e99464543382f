"""Pins of the reference MLP (binary64): the backward pass against central
finite differences, the encoding against its definition at special points,
and the rounding helper against exact bfloat16 values."""
import numpy as np

from oracle import mlp_ref as M


def test_param_count():
    assert M.N_PARAMS == 14544
    # 80*64 + 64 + 2*(64*64 + 64) + 16*64 + 16 = 13.7k real + padding


def test_bf16_rounding_exact_cases():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0], np.float32)
    r = M.bf16(x)
    # ties to even: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6
    np.testing.assert_array_equal(r, [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 0.0])


def test_encoding_special_points():
    f = M.encode(np.array([[0.0, 0.5, 1.0, -1.0, 0.25, 0.0]]))
    # dim 0 at x = 0: sin = 0, cos = 1 for every frequency
    np.testing.assert_allclose(f[0, 0:12:2], 0.0, atol=1e-15)
    np.testing.assert_allclose(f[0, 1:12:2], 1.0)
    # dim 1 at x = 0.5, k = 0: sin(pi/2) = 1, cos = 0; k = 1: sin(pi) = 0, cos = -1
    np.testing.assert_allclose(f[0, 12:16], [1.0, 0.0, 0.0, -1.0], atol=1e-15)
    assert np.all(f[0, 72:] == 0)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    flat = M.init_params(3).astype(np.float64)
    x = np.concatenate([rng.random((9, 3)), rng.uniform(-1, 1, (9, 3))], 1)
    tgt = rng.normal(size=(9, 3))
    w = rng.random((9, 3))
    _, g = M.loss_and_grad(flat, x, tgt, w, bf16_round=False)
    idx = np.concatenate([rng.choice(M.N_PARAMS - 2000, 60, replace=False),
                          np.arange(M.N_PARAMS - 1104, M.N_PARAMS - 1104 + 3 * 64, 7)])
    for i in idx:
        h = 1e-6
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp, _ = M.loss_and_grad(fp, x, tgt, w, bf16_round=False)
        lm, _ = M.loss_and_grad(fm, x, tgt, w, bf16_round=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_padding_gradient_is_zero():
    rng = np.random.default_rng(1)
    flat = M.init_params(5).astype(np.float64)
    x = np.concatenate([rng.random((7, 3)), rng.uniform(-1, 1, (7, 3))], 1)
    _, g = M.loss_and_grad(flat, x, rng.normal(size=(7, 3)), rng.random((7, 3)))
    p = M.unpack(g)
    assert np.all(p["W4"][3:] == 0) and np.all(p["b4"][3:] == 0)


def test_adam_matches_definition_first_step():
    g = np.array([0.5, -2.0, 0.0], np.float32)
    w, m, v = M.adam_step(np.zeros(3, np.float32), g, np.zeros(3), np.zeros(3), 1, lr=1e-3)
    # first step: m_hat = g, v_hat = g^2, so the update is -lr * sign(g) (eps aside)
    np.testing.assert_allclose(w, [-1e-3, 1e-3, 0.0], rtol=1e-5, atol=1e-12)
