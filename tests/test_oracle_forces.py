"""Pins for the oracle's per-pair forces and loss terms.

The forces are checked against torch autograd of the per-vertex loss of Eq. 2
written from the similarity functions alone (sigmoid of the dot product,
Eq. 3; Student-t kernel 1/(1+t^2), Eq. 7), so a dropped term, a sign error or
a wrong direction vector in the hand-derived gradients (Eqs. 5-6, 8-9) fails.
The loss terms are checked against scipy's log-sigmoid and against special
values."""
import numpy as np
import pytest
import torch
from scipy import special

import oracle


def autograd_vertex_grad(force, eps, zu, nbrs, negs):
    z = torch.tensor(zu, dtype=torch.float64, requires_grad=True)
    N = torch.tensor(np.asarray(nbrs).reshape(-1, len(zu)), dtype=torch.float64)
    S = torch.tensor(np.asarray(negs).reshape(-1, len(zu)), dtype=torch.float64)
    if force == "sigmoid":
        # log delta and log(1 - delta) through log-sigmoid (1 - sigma(x) = sigma(-x))
        # so the reference value itself keeps full precision for large |x|
        L = -torch.nn.functional.logsigmoid(N @ z).sum() - torch.nn.functional.logsigmoid(-(S @ z)).sum()
    else:
        tn2 = ((z[None, :] - N) ** 2).sum(1)
        ts2 = ((z[None, :] - S) ** 2).sum(1)
        delta_n = 1.0 / (1.0 + tn2)
        delta_s = (1.0 - eps) / (1.0 + ts2)   # eps = 0 is the paper's kernel
        L = -torch.log(delta_n).sum() - torch.log(1 - delta_s).sum()
    L.backward()
    return z.grad.numpy(), float(L)


@pytest.mark.parametrize("force", ["sigmoid", "student_t"])
@pytest.mark.parametrize("eps", [0.0, 1e-3, 0.1])
@pytest.mark.parametrize("d", [1, 2, 7, 32])
def test_gradient_matches_autograd(force, eps, d):
    if force == "sigmoid" and eps != 1e-3:
        pytest.skip("eps only enters the Student-t model")
    rng = np.random.default_rng(d * 7 + int(eps * 1000))
    for trial in range(5):
        zu = rng.normal(size=d)
        nbrs = rng.normal(size=(rng.integers(0, 6), d))
        negs = rng.normal(size=(rng.integers(0, 6), d))
        g = oracle.vertex_gradient(force, eps, zu, nbrs, negs)
        ga, L = autograd_vertex_grad(force, eps, zu, nbrs, negs)
        np.testing.assert_allclose(g, ga, rtol=1e-11, atol=1e-12)
        assert oracle.pair_losses(force, eps, zu, nbrs, negs) == pytest.approx(L, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("force", ["sigmoid", "student_t"])
def test_gradient_finite_difference(force):
    rng = np.random.default_rng(5)
    d, h, eps = 6, 1e-6, 1e-3
    zu = rng.normal(size=d)
    nbrs = rng.normal(size=(4, d))
    negs = rng.normal(size=(3, d))
    g = oracle.vertex_gradient(force, eps, zu, nbrs, negs)
    fd = np.zeros(d)
    for i in range(d):
        e = np.zeros(d)
        e[i] = h
        fd[i] = (oracle.pair_losses(force, eps, zu + e, nbrs, negs)
                 - oracle.pair_losses(force, eps, zu - e, nbrs, negs)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-7, atol=1e-8)


def test_sigmoid_loss_terms_match_scipy():
    rng = np.random.default_rng(9)
    for _ in range(50):
        a, c = rng.normal(size=8) * 3, rng.normal(size=8) * 3
        x = a @ c
        assert oracle.pair_loss("sigmoid", 0.0, a, c, False) == pytest.approx(-special.log_expit(x), rel=1e-12)
        assert oracle.pair_loss("sigmoid", 0.0, a, c, True) == pytest.approx(-special.log_expit(-x), rel=1e-12)
    # large |x|: stable, no overflow
    a = np.array([30.0, 0.0])
    c = np.array([30.0, 0.0])
    assert oracle.pair_loss("sigmoid", 0.0, a, c, True) == pytest.approx(900.0, rel=1e-12)
    assert oracle.pair_loss("sigmoid", 0.0, a, c, False) == pytest.approx(np.exp(-900.0), abs=1e-300)


def test_student_t_loss_special_values():
    a = np.array([0.3, -0.2, 0.5])
    # coincident rows: -log delta = 0; repulsion -log(1 - (1-eps)) = -log(eps)
    assert oracle.pair_loss("student_t", 1e-3, a, a, False) == 0.0
    assert oracle.pair_loss("student_t", 1e-3, a, a, True) == pytest.approx(-np.log(1e-3), rel=1e-12)
    # unit distance: -log(1/2) and -log(1/2) (eps = 0)
    c = a + np.array([1.0, 0.0, 0.0])
    assert oracle.pair_loss("student_t", 0.0, a, c, False) == pytest.approx(np.log(2.0), rel=1e-14)
    assert oracle.pair_loss("student_t", 0.0, a, c, True) == pytest.approx(np.log(2.0), rel=1e-14)
    # sigmoid at orthogonal rows: log 2 both ways
    assert oracle.pair_loss("sigmoid", 0.0, np.array([1.0, 0]), np.array([0, 1.0]), False) == pytest.approx(np.log(2))


def test_repulsion_from_self_is_zero_for_student_t():
    a = np.array([0.1, 0.2, -0.3])
    for eps in (0.0, 1e-3):
        g = oracle.vertex_gradient("student_t", eps, a, np.zeros((0, 3)), a[None, :])
        assert np.all(g == 0.0)


def test_forces_point_the_right_way():
    # attraction pulls u towards v (descent direction -g points to c), repulsion pushes away
    a = np.array([0.0, 0.0])
    c = np.array([1.0, 0.0])
    ga = oracle.vertex_gradient("student_t", 1e-3, a, c[None, :], np.zeros((0, 2)))
    gr = oracle.vertex_gradient("student_t", 1e-3, a, np.zeros((0, 2)), c[None, :])
    assert (-ga) @ (c - a) > 0 and (-gr) @ (c - a) < 0
    # sigmoid: attraction increases the dot product, repulsion decreases it
    a = np.array([0.2, 0.1])
    ga = oracle.vertex_gradient("sigmoid", 0.0, a, c[None, :], np.zeros((0, 2)))
    gr = oracle.vertex_gradient("sigmoid", 0.0, a, np.zeros((0, 2)), c[None, :])
    assert (-ga) @ c > 0 and (-gr) @ c < 0


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=20000).astype(np.float32),
                        (rng.normal(size=2000) * 1e-30).astype(np.float32),
                        np.array([1 + 2**-8, 1 + 3 * 2**-8, -(1 + 2**-8), 0.0, 65504.0], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    mine = np.array([oracle.bf16_round(float(v)) for v in x])
    # torch rounds subnormal bf16 results the same way for normal float32 input
    np.testing.assert_array_equal(mine, ref)
