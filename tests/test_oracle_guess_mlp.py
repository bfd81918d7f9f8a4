"""Pins of the start-vector estimators (Sec. IV, eq. (4)-(5)) and of the FP64
network reference (CPU only)."""

import numpy as np
import pytest

import eqsgen
from oracle import guess, mlp
from oracle.eqs import EqsOracle


def test_mgs_orthonormal_and_span():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(200, 6))
    X[:, 4] = 2 * X[:, 1] - X[:, 3]  # dependent column is dropped
    V = guess.mgs(X)
    assert V.shape == (200, 5)
    np.testing.assert_allclose(V.T @ V, np.eye(5), atol=1e-13)
    P = V @ V.T
    np.testing.assert_allclose(P @ X, X, atol=1e-12 * np.abs(X).max())


def test_galerkin_exact_for_solution_in_span():
    """P10: if the stage solution lies in span(V), eq. (5) returns it exactly."""
    case = eqsgen.case_c1(n=6, seed=1)
    o = EqsOracle(case)
    rng = np.random.default_rng(1)
    ystar = rng.normal(size=o.n_free)
    b = o.M_II @ ystar
    V = guess.mgs(np.column_stack([rng.normal(size=o.n_free), ystar, rng.normal(size=o.n_free)]))
    x0 = guess.galerkin_start(V, o.M_II, b)
    np.testing.assert_allclose(x0, ystar, atol=1e-10 * np.abs(ystar).max())


def test_galerkin_is_energy_optimal():
    """The error of eq. (5) is M-orthogonal to span(V), so no other guess in
    span(V) has a smaller M-norm error."""
    case = eqsgen.case_c1(n=6, seed=2)
    o = EqsOracle(case)
    rng = np.random.default_rng(2)
    b = rng.normal(size=o.n_free)
    xs = o.solve(b)
    V = guess.mgs(rng.normal(size=(o.n_free, 5)))
    x0 = guess.galerkin_start(V, o.M_II, b)
    e = xs - x0
    assert np.abs(V.T @ (o.M_II @ e)).max() <= 1e-10 * np.abs(V.T @ (o.M_II @ xs)).max()
    enorm = lambda v: np.sqrt(v @ (o.M_II @ v))
    for _ in range(5):
        other = x0 + V @ rng.normal(scale=1e-2 * np.linalg.norm(x0), size=V.shape[1])
        assert enorm(xs - other) > enorm(e)


def test_pod_gram_route_equals_svd():
    rng = np.random.default_rng(3)
    S = rng.normal(size=(500, 16)) @ np.diag(np.logspace(0, -5, 16))
    V1, s1 = guess.pod_basis(S, 16)
    V2, s2, W = guess.pod_from_gram(S, 16)
    np.testing.assert_allclose(s2, s1, rtol=1e-9)
    np.testing.assert_allclose(V2 @ V2.T, V1 @ V1.T, atol=1e-8)
    # rank-deficient snapshots: the Gram route keeps only resolvable directions
    S[:, 10:] = S[:, :6] @ rng.normal(size=(6, 6))
    V3, s3, _ = guess.pod_from_gram(S, 16)
    assert V3.shape[1] == 10
    np.testing.assert_allclose(V3.T @ V3, np.eye(10), atol=1e-6)


def _params(seed):
    return {k: v.astype(np.float64) for k, v in eqsgen.mlp_init(seed).items()}


def test_mlp_gradients_central_differences():
    """P11: FP64 backward vs central differences (h = 1e-6, rel <= 1e-6)."""
    p = _params(4)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(8, 32))
    t = rng.normal(size=(8, 16))
    L, g = mlp.backward(p, x, t)
    assert L == pytest.approx(mlp.loss(p, x, t), rel=1e-15)
    h = 1e-6
    for k in mlp.NAMES:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = mlp.loss(p, x, t)
            flat[i] = old - h
            lm = mlp.loss(p, x, t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            # 1e-6 relative, above the difference quotient's rounding floor eps*L/h ~ 1e-10
            assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (k, i, fd, an)


def test_adam_first_step_is_signed_lr():
    """Adam's bias correction makes the first step exactly lr * sign(g) (up to eps)."""
    p = _params(6)
    rng = np.random.default_rng(7)
    x, t = rng.normal(size=(16, 32)), rng.normal(size=(16, 16))
    _, g = mlp.backward(p, x, t)
    q = {k: v.copy() for k, v in p.items()}
    st = mlp.adam_state(q)
    mlp.adam_step(q, g, st, lr=1e-3)
    for k in mlp.NAMES:
        big = np.abs(g[k]) > 1e-4
        np.testing.assert_allclose((p[k] - q[k])[big], 1e-3 * np.sign(g[k][big]), rtol=1e-3)


def test_training_reduces_loss_on_linear_map():
    """The network learns a linear map of its inputs (the Galerkin coefficients
    are linear in the projected right-hand side)."""
    p = _params(8)
    rng = np.random.default_rng(9)
    A = rng.normal(size=(16, 32)) / 6
    st = mlp.adam_state(p)
    X = rng.normal(size=(512, 32))
    Y = X @ A.T
    l0 = mlp.loss(p, X, Y)
    for it in range(400):
        b = rng.choice(512, 64, replace=False)
        _, g = mlp.backward(p, X[b], Y[b])
        mlp.adam_step(p, g, st)
    assert mlp.loss(p, X, Y) < 0.05 * l0


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(10)
    a = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-8, 8, 2000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0, -0.0])])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.round_bf16(a), ref)


def _torch_net(p, bf16):
    """The network written out in torch float64 (an implementation independent
    of the oracle's): torch's SiLU, explicit products, torch's bfloat16
    conversion for the BF16 form's operands."""
    torch = pytest.importorskip("torch")
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}

    def q(a):
        return a.to(torch.float32).to(torch.bfloat16).to(torch.float64) if bf16 else a

    def fwd(x):
        a1 = torch.nn.functional.silu(torch.mm(q(x), q(P["W1"]).t()) + P["b1"])
        a2 = torch.nn.functional.silu(torch.mm(q(a1), q(P["W2"]).t()) + P["b2"])
        return torch.mm(q(a2), q(P["W3"]).t()) + P["b3"]

    return P, fwd


@pytest.mark.parametrize("bf16", [False, True])
def test_mlp_forward_matches_torch_float64(bf16):
    """The oracle's forward (both forms) equals the network written in torch."""
    torch = pytest.importorskip("torch")
    p = _params(11)
    rng = np.random.default_rng(12)
    x = rng.normal(size=(40, 32)) * 2.0
    _, fwd = _torch_net(p, bf16)
    ref = fwd(torch.tensor(x)).detach().numpy()
    y, _ = mlp.forward(p, x, bf16=bf16)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    if bf16:
        # the rounding matters: the BF16 form differs from the FP64 network
        y64, _ = mlp.forward(p, x)
        assert np.abs(y - y64).max() > 1e-4 * np.abs(y64).max()


def test_mlp_gradients_match_torch_autograd():
    """The oracle's backward equals torch's automatic differentiation of the
    mean-squared error of the same network, in float64."""
    torch = pytest.importorskip("torch")
    p = _params(13)
    rng = np.random.default_rng(14)
    x, t = rng.normal(size=(24, 32)), rng.normal(size=(24, 16))
    P, fwd = _torch_net(p, False)
    L = torch.mean((fwd(torch.tensor(x)) - torch.tensor(t)) ** 2)
    L.backward()
    Lo, g = mlp.backward(p, x, t)
    assert Lo == pytest.approx(L.item(), rel=1e-14)
    for k in mlp.NAMES:
        ref = P[k].grad.numpy()
        np.testing.assert_allclose(g[k], ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_mlp_bf16_gradients_near_exact_ones():
    """The BF16 form's gradients (products of rounded operands) stay within a
    few bfloat16 unit roundoffs (2^-8) of the exact gradients."""
    p = _params(15)
    rng = np.random.default_rng(16)
    x, t = rng.normal(size=(64, 32)), rng.normal(size=(64, 16))
    _, g = mlp.backward(p, x, t)
    _, gb = mlp.backward(p, x, t, bf16=True)
    for k in mlp.NAMES:
        r = np.linalg.norm(gb[k] - g[k]) / np.linalg.norm(g[k])
        assert 1e-5 < r < 4 * 2.0 ** -8, (k, r)


def test_adam_matches_torch_optimizer():
    """Five Adam steps of the oracle equal torch.optim.Adam in float64 with the
    same gradients (lr 1e-3, betas 0.9 / 0.999, eps 1e-8)."""
    torch = pytest.importorskip("torch")
    p = _params(17)
    rng = np.random.default_rng(18)
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam([P[k] for k in mlp.NAMES], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    q = {k: v.copy() for k, v in p.items()}
    st = mlp.adam_state(q)
    for _ in range(5):
        g = {k: rng.normal(size=v.shape) * 10.0 ** rng.uniform(-6, 0) for k, v in p.items()}
        for k in mlp.NAMES:
            P[k].grad = torch.tensor(g[k])
        opt.step()
        mlp.adam_step(q, g, st, lr=1e-3)
    for k in mlp.NAMES:
        np.testing.assert_allclose(q[k], P[k].detach().numpy(), rtol=0, atol=1e-14)
