"""Pins of the oracle MLP: finite-difference gradients, linear special case,
Adam's closed-form first step."""
import numpy as np
import pytest

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


def test_features_of_a_hand_built_box():
    """Every named feature of a box whose values are fixed by hand: V takes
    -2, -1, 1, 2 on six points each (min -2, max 2, mean 0, std sqrt(2.5);
    histogram bins 0, 8, 24 and 31 each hold a quarter), two atoms with known
    gammas, a 1 x 1 x 2 core in a 2 x 3 x 4 box."""
    from types import SimpleNamespace
    v = np.repeat([-2.0, -1.0, 1.0, 2.0], 6)
    proj = np.array([[2.0, 0.5, 1.0, -0.5, 0.25, 0.25], [2.0, 0.5, 0.5, 0.1, 0.1, 0.1]])
    sd = SimpleNamespace(v=v, n=(2, 3, 4), h=0.4275, core_lo=(1, 1, 1), core_hi=(2, 2, 3),
                         atoms=np.zeros((2, 3)), ns=5, proj=proj)
    f = mlp.features(sd)
    hist = np.zeros(32)
    hist[[0, 8, 24, 31]] = 0.25
    assert np.array_equal(f[:32], hist)
    named = [2, 2, 3, 4, 0.4275, 0.4275, -2.0, 2.0, 0.0, np.sqrt(2.5), 5, 8, 2.8, 2 / 24]
    assert np.allclose(f[32:46], named, rtol=1e-14, atol=1e-15)
    # the closed-form top of -1/2 Lap: 1.5 * 7.0729389 / h^2 = 58.0522 Ha at this h
    assert f[46] == pytest.approx(58.0522, abs=5e-5)
    assert np.all(f[47:] == 0.0)


def test_lap_lambda_max_equals_brute_force_top_eigenvalue():
    """The closed-form largest eigenvalue of -1/2 Lap (periodic; theta = pi on
    every axis) equals the top eigenvalue of the dense operator on an even
    periodic grid."""
    from types import SimpleNamespace
    from oracle import hamiltonian
    h = 0.61
    op = hamiltonian.free_operator((8, 8, 8), h, True)
    top = np.linalg.eigvalsh(op.dense())[-1]
    assert mlp.lap_lambda_max(SimpleNamespace(h=h)) == pytest.approx(top, rel=1e-12)
