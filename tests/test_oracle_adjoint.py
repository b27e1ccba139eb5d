"""Pins of the oracle's differentiable form (adjoint along a fixed trajectory).

With every key, count, weight and merge group fixed, the modes are a linear
function of the points (Eq. 1-4 with constant discrete structure), with the
same weights for every coordinate: mu_c = sum_i J_ci x_i.  Pinned by:
* the exact-rational Jacobian of a brute force (tests/exact_reference.py);
* closed forms: with no round executed, J_ci = 1/C_c for the points of c;
* invariants: J >= 0 and every row sums to 1 (a mode is a weighted average of
  points, so translating all points translates every mode);
* central finite differences of the point-to-mode loss evaluated in binary128
  along the same trajectory, at perturbations whose FP64 fits are checked to
  follow the identical discrete path;
* the loss value and the per-cluster point sums against exact summation.
"""
import math

import numpy as np
import pytest

from exact_reference import exact_jacobian
from paper_2206_02200_amd import synth


def _small(seed, n=None, d=None):
    rng = np.random.default_rng(seed)
    d = d or int(rng.integers(1, 4))
    n = n or int(rng.integers(4, 30))
    k = int(rng.integers(1, 4))
    c = rng.uniform(0, 8, size=(k, d))
    x = c[rng.integers(0, k, size=n)] + 1.1 * rng.standard_normal(size=(n, d))
    return synth.dyadic(x, bits=10), float(rng.choice([0.5, 1.0, 2.0]))


@pytest.mark.parametrize("seed", list(range(500, 530)))
def test_adjoint_matches_exact_jacobian(oracle, seed):
    x, h = _small(seed)
    J, margin = exact_jacobian(x, h, max_iter=40)
    if margin is not None and margin < 1e-9:
        pytest.skip("a floor decision sits within rounding of a cell boundary")
    res, tape = oracle.fit_tape(x, h, 40)
    Jf = np.array([[float(v) for v in row] for row in J])
    assert Jf.shape == (res.K, len(x))
    # invariants of the exact Jacobian
    assert np.all(Jf >= 0)
    np.testing.assert_allclose(Jf.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    rng = np.random.default_rng(seed)
    mubar = rng.standard_normal(size=(res.K, x.shape[1]))
    got = tape.point_adjoint(mubar)
    want = Jf.T @ mubar
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13 * np.abs(mubar).max())
    # the modes themselves are J x
    np.testing.assert_allclose(res.modes, Jf @ x, rtol=1e-12, atol=1e-12)


def test_no_round_gives_cell_means(oracle):
    x = np.array([[0.5, 0.5], [0.7, 0.2], [3.5, 3.5], [3.25, 3.75], [3.6, 3.1]])
    res, tape = oracle.fit_tape(x, 1.0)
    assert res.n_iter == 0
    mubar = np.array([[1.0, -2.0], [0.5, 4.0]])
    g = tape.point_adjoint(mubar)
    want = np.array([mubar[res.labels[i]] / res.counts[res.labels[i]] for i in range(len(x))])
    np.testing.assert_array_equal(g, want)


def test_worked_example_gradient_by_hand(oracle):
    # A1: x = [0.5, 1.25, 1.75, 2.5], one round, mode = ((1*p0 + 2*p1) + 1*p2)/4
    # with p0 = (x0 + (x1+x2))/3, p1 = (x0 + (x1+x2) + x3)/4, p2 = ((x1+x2) + x3)/3
    # d mode / dx0 = (1/3 + 2/4)/4, dx1 = dx2 = (1/3 + 2/4 + 1/3)/4, dx3 = (2/4 + 1/3)/4
    x = np.array([[0.5], [1.25], [1.75], [2.5]])
    res, tape = oracle.fit_tape(x, 1.0)
    g = tape.point_adjoint(np.array([[1.0]])).ravel()
    want = [(1 / 3 + 2 / 4) / 4, (1 / 3 + 2 / 4 + 1 / 3) / 4, (1 / 3 + 2 / 4 + 1 / 3) / 4, (2 / 4 + 1 / 3) / 4]
    np.testing.assert_allclose(g, want, rtol=1e-15)
    assert abs(sum(want) - 1.0) < 1e-15


@pytest.mark.parametrize("seed", [601, 602, 603, 604])
def test_loss_gradient_against_binary128_finite_differences(oracle, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.normal(c, 1.3, size=(60, 3)) for c in ([0, 0, 0], [6, 1, 2], [2, 7, 5])])
    h = 1.5
    L, grad, res, tape = oracle.loss_and_grad(x, h)
    assert res.n_iter >= 1
    eps = 1e-4
    checked = 0
    for i in rng.choice(len(x), size=12, replace=False):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += eps
            xm[i, k] -= eps
            _, tp = oracle.fit_tape(xp, h)
            _, tm = oracle.fit_tape(xm, h)
            if not (tape.same_trajectory(tp) and tape.same_trajectory(tm)):
                continue  # the perturbation crossed a cell boundary somewhere
            fd = tape.fd_q(x, i, k, eps)
            assert abs(fd - grad[i, k]) <= 1e-9 * max(1.0, abs(fd)), (i, k, fd, grad[i, k])
            checked += 1
    assert checked >= 20


def test_loss_value_and_cluster_sums(oracle):
    rng = np.random.default_rng(611)
    x = rng.normal(0, 3, size=(400, 2))
    res, tape = oracle.fit_tape(x, 2.0)
    L = oracle.point_mode_loss(x, res.labels, res.modes)
    exact = math.fsum(float(((x[i] - res.modes[res.labels[i]]) ** 2).sum()) for i in range(len(x)))
    assert abs(L - exact) <= 1e-13 * exact
    X = tape.cluster_point_sums()
    for c in range(res.K):
        for k in range(2):
            assert abs(X[c, k] - math.fsum(x[res.labels == c, k])) <= 1e-12 * (1 + np.abs(x[:, k]).sum())
    # the replayed (binary128) loss along the trajectory equals the FP64 loss
    assert abs(tape.replay_loss(x) - L) <= 1e-12 * L
