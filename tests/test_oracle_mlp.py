"""Pins of the oracle MLP: finite-difference gradients, linear special case,
Adam's closed-form first step."""
import numpy as np

from oracle import mlp
from paper_2609_13115_amd import workloads


def _params(sizes, seed=0):
    return workloads.mlp_init(sizes, seed)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    sizes = (6, 5, 4, 3)
    P = _params(sizes)
    X = rng.standard_normal((7, 6))
    T = rng.standard_normal((7, 3))
    Y, cache = mlp.forward(P, X)
    G = mlp.backward(P, cache, Y, T)
    eps = 1e-6
    for i, p in enumerate(P):
        it = np.nditer(p, flags=["multi_index"])
        for _ in it:
            k = it.multi_index
            old = p[k]
            p[k] = old + eps
            lp = mlp.mse(mlp.forward(P, X)[0], T)
            p[k] = old - eps
            lm = mlp.mse(mlp.forward(P, X)[0], T)
            p[k] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - G[i][k]) <= 1e-6 * max(1.0, abs(fd)), (i, k, fd, G[i][k])


def test_linear_model_converges_to_least_squares():
    """No hidden layer: Adam on the MSE reaches numpy.linalg.lstsq."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((200, 5))
    Wt = rng.standard_normal((5, 2))
    T = X @ Wt + 0.3 + 0.01 * rng.standard_normal((200, 2))
    P = [np.zeros((5, 2)), np.zeros(2)]
    batches = [np.arange(200)] * 6000
    P, losses = mlp.train(P, X, T, batches, lr=1e-2)
    Xa = np.hstack([X, np.ones((200, 1))])
    sol, *_ = np.linalg.lstsq(Xa, T, rcond=None)
    assert np.allclose(P[0], sol[:5], atol=1e-4)
    assert np.allclose(P[1], sol[5], atol=1e-4)


def test_adam_first_step_closed_form():
    P = [np.array([[1.0, -2.0]]), np.array([0.5, 0.0])]
    G = [np.array([[0.3, -4.0]]), np.array([1e-3, 0.0])]
    st = mlp.adam_init(P)
    out = mlp.adam_step(P, G, st, lr=0.1)
    for p, g, o in zip(P, G, out):
        assert np.allclose(o, p - 0.1 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_features_shape_and_histogram():
    sd = workloads.small_dirichlet(ns=4)
    f = mlp.features(sd)
    assert f.shape == (64,)
    assert abs(f[:32].sum() - 1.0) < 1e-12
    assert f[32] == len(sd.atoms)
    assert abs(f[46] - 1.5 * 7.0729389 / sd.h ** 2) < 1e-5 * f[46]
