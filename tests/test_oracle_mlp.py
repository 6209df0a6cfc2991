"""Pins of the FP64 proposal-network reference (oracle/mlp.py)."""
import numpy as np

from oracle import mlp as M
from paper_2501_05828_amd import scenes


def _setup(rows=6, seed=0):
    rng = np.random.default_rng(seed)
    xn, tn = M.row_inputs(2, rows // 2, 0.3e-3, np.deg2rad([-10.0, 10.0]))
    B = rng.normal(size=(M.N_RFF, 2))
    X = M.features(xn, tn, B)
    H = rng.gamma(0.3, size=(rows, M.N_OUT)) * (rng.uniform(size=(rows, M.N_OUT)) < 0.05)
    H[:, 7] += 1.0
    theta = scenes.proposal_init(seed)[0].astype(np.float64)
    theta += rng.normal(0, 0.01, size=theta.shape)       # non-zero biases too
    return X, H, theta


def test_parameter_count():
    assert M.N_PARAMS == 77120


def test_features_are_bounded_and_periodic():
    xn, tn = M.row_inputs(3, 128, 0.3e-3, np.deg2rad([-20.0, 0.0, 20.0]))
    assert xn.min() > -1 and xn.max() < 1 and tn.min() == -1 and tn.max() == 1
    X = M.features(xn, tn, np.ones((16, 2)))
    assert X.shape == (384, 34)
    assert np.allclose(X[:, 2:18] ** 2 + X[:, 18:] ** 2, 1.0)


def test_gradient_matches_central_differences():
    X, H, theta = _setup()
    _, g = M.loss_and_grad(theta, X, H, q_bf16=False)
    rng = np.random.default_rng(1)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SHAPES])
    idx = np.concatenate([rng.integers(offs[i], offs[i + 1], 6) for i in range(len(M.SHAPES))])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.loss_and_grad(tp, X, H, False)[0] - M.loss_and_grad(tm, X, H, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_softmax_and_one_hot_loss():
    X, _, theta = _setup()
    f = M.forward(theta, X, q_bf16=False)
    assert np.allclose(f["q"].sum(1), 1.0)
    H = np.zeros((X.shape[0], M.N_OUT))
    H[0, 123] = 2.5
    loss, _ = M.loss_and_grad(theta, X, H, q_bf16=False)
    assert abs(loss + np.log(f["q"][0, 123])) < 1e-12


def test_stationary_at_target_distribution():
    """With W4 = 0 and b4 = log of the normalised target row, q equals the
    target and the loss gradient with respect to b4 vanishes."""
    X, H, theta = _setup(rows=2)
    H = H[:1].copy()
    H[0] += 0.01
    X = X[:1]
    p = M.unpack(theta)
    p["W4"][:] = 0.0
    p["b4"][:] = np.log(H[0] / H[0].sum())
    theta = M.pack(p)
    f = M.forward(theta, X, q_bf16=False)
    assert np.allclose(f["q"][0], H[0] / H[0].sum(), rtol=1e-12)
    _, g = M.loss_and_grad(theta, X, H, q_bf16=False)
    gb4 = M.unpack(g)["b4"]
    assert np.max(np.abs(gb4)) < 1e-15


def test_adam_first_step_is_signed_learning_rate():
    rng = np.random.default_rng(2)
    th = rng.normal(size=100)
    g = rng.normal(size=100)
    new, m, v = M.adam(th, g, np.zeros(100), np.zeros(100), 1, 1e-3)
    assert np.allclose(new - th, -1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.0, 1.0 + 2 ** -7 + 2 ** -8, 0.0], np.float32)
    want = np.array([1.0, 1.0, 1.0 + 2 ** -7, -3.0, 1.0 + 2 ** -6, 0.0])
    assert np.array_equal(M.bf16(vals), want)


def test_bf16_loss_close_to_exact():
    X, H, theta = _setup()
    l16, g16 = M.loss_and_grad(theta, X, H, True)
    l64, g64 = M.loss_and_grad(theta, X, H, False)
    assert abs(l16 - l64) < 2e-2 * abs(l64)
    assert np.linalg.norm(g16 - g64) < 0.15 * np.linalg.norm(g64)


def test_proposal_tables():
    q = np.random.default_rng(3).dirichlet(np.ones(1024), size=4)
    qm, cdf = M.proposal_tables(q, 0.1)
    assert np.all(qm >= 0.1 / 1024 - 1e-18)
    assert np.allclose(cdf[:, -1], 1.0)
    assert np.all(np.diff(cdf, axis=1) > 0)
