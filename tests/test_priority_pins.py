"""Pins of the learned-priority oracle (CPU): the gradient against central
finite differences and against torch's autograd in float64, closed forms of the
network and of the loss, the first two Adam steps in closed form and five steps
against torch.optim.Adam, and the feature and schedule definitions on
hand-checked cases."""
import numpy as np
import pytest

from oracle import priority as P


def _random_problem(seed, n=24, scale=0.5):
    rng = np.random.default_rng(seed)
    params = rng.normal(0, scale, P.N_PARAMS)
    x = rng.normal(0, 1, (n, P.N_FEATURES))
    y = (rng.random(n) < 0.4).astype(np.float64)
    return params, x, y


def test_parameter_count_and_layout():
    assert P.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5057
    params = np.arange(P.N_PARAMS, dtype=np.float64)
    parts = P.unpack(params)
    assert parts["W1"][0, 1] == 1 and parts["W1"][1, 0] == 64  # input-major
    assert parts["b1"][0] == 768 and parts["W2"][0, 0] == 832 and parts["b2"][0] == 4928
    assert parts["w3"][0] == 4992 and parts["b3"][0] == 5056
    np.testing.assert_array_equal(P.pack(parts), params)


def test_gradient_matches_central_differences():
    params, x, y = _random_problem(1)
    _, g = P.loss_grad(params, x, y)
    h = 1e-6
    num = np.empty(P.N_PARAMS)
    for i in range(P.N_PARAMS):
        e = np.zeros(P.N_PARAMS)
        e[i] = h
        num[i] = (P.loss(params + e, x, y) - P.loss(params - e, x, y)) / (2 * h)
    assert np.max(np.abs(num - g)) < 1e-7 * max(1.0, np.max(np.abs(g))) + 1e-9


def test_forward_and_gradient_match_torch_autograd():
    torch = pytest.importorskip("torch")
    params, x, y = _random_problem(2, n=40)
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.unpack(params).items()}
    xt, yt = torch.tensor(x), torch.tensor(y)
    h1 = torch.relu(xt @ t["W1"] + t["b1"])
    h2 = torch.relu(h1 @ t["W2"] + t["b2"])
    z3 = h2 @ t["w3"] + t["b3"][0]
    lt = torch.nn.functional.binary_cross_entropy_with_logits(z3, yt)
    lt.backward()
    value, g = P.loss_grad(params, x, y)
    np.testing.assert_allclose(P.forward(params, x)["prob"], torch.sigmoid(z3).detach().numpy(), rtol=1e-12)
    assert abs(value - lt.item()) < 1e-12
    np.testing.assert_allclose(g, P.pack({k: v.grad.numpy() for k, v in t.items()}), atol=1e-12)


def test_closed_forms():
    x = np.random.default_rng(3).normal(size=(7, 12))
    zero = np.zeros(P.N_PARAMS)
    np.testing.assert_allclose(P.forward(zero, x)["prob"], 0.5)
    assert abs(P.loss(zero, x, np.array([0, 1, 1, 0, 1, 0, 0.0])) - np.log(2)) < 1e-15
    only_b3 = zero.copy()
    only_b3[-1] = 1.3
    np.testing.assert_allclose(P.forward(only_b3, x)["prob"], 1 / (1 + np.exp(-1.3)))
    # softplus form equals the textbook cross-entropy
    y = np.array([1, 0, 1, 0, 1, 0, 1.0])
    p = 1 / (1 + np.exp(-1.3))
    want = -np.mean(y * np.log(p) + (1 - y) * np.log(1 - p))
    assert abs(P.loss(only_b3, x, y) - want) < 1e-14
    # the gradient of the last bias alone is mean(p - y)
    _, g = P.loss_grad(only_b3, x, y)
    assert abs(g[-1] - np.mean(p - y)) < 1e-15
    assert np.all(g[:-1] == 0)  # relu(0) = 0 and its derivative is taken as 0


def test_first_adam_step_closed_form():
    params, x, y = _random_problem(4)
    _, g = P.loss_grad(params, x, y)
    lr, eps = 1e-2, 1e-8
    theta, losses = P.adam(params, x, y, [np.arange(len(y))], lr=lr, eps=eps)
    # bias-corrected moments of one step are g and g^2
    np.testing.assert_allclose(theta, params - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    assert losses.shape == (1,)


def test_two_adam_steps_closed_form():
    """Two steps with unequal moment decays: after gradients g1 then g2 the
    moments are m = b1 (1 - b1) g1 + (1 - b1) g2 and v = b2 (1 - b2) g1^2 +
    (1 - b2) g2^2, divided by 1 - b1^2 and 1 - b2^2 before the step.  Swapping
    the two decays changes the result, unlike the first step."""
    params, x, y = _random_problem(5)
    lr, b1, b2, eps = 3e-3, 0.8, 0.95, 1e-7
    idx = [np.arange(0, 12), np.arange(12, 24)]
    _, g1 = P.loss_grad(params, x[idx[0]], y[idx[0]])
    theta1 = params - lr * g1 / (np.abs(g1) + eps)
    _, g2 = P.loss_grad(theta1, x[idx[1]], y[idx[1]])
    m = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    v = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    want = theta1 - lr * m / (np.sqrt(v) + eps)
    got, losses = P.adam(params, x, y, idx, lr=lr, beta1=b1, beta2=b2, eps=eps)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)
    assert losses.shape == (2,)
    swapped, _ = P.adam(params, x, y, idx, lr=lr, beta1=b2, beta2=b1, eps=eps)
    assert np.max(np.abs(swapped - want)) > 1e-6


def test_adam_matches_torch_optim_over_several_steps():
    """Five minibatch steps with non-default decays against torch.optim.Adam in
    float64, the gradient of each step taken by torch's autograd."""
    torch = pytest.importorskip("torch")
    params, x, y = _random_problem(6, n=40)
    lr, b1, b2, eps = 5e-3, 0.7, 0.9, 1e-6
    batches = [np.arange(i, 40, 5) for i in range(5)]
    got, losses = P.adam(params, x, y, batches, lr=lr, beta1=b1, beta2=b2, eps=eps)
    t = {k: torch.tensor(v.copy(), dtype=torch.float64, requires_grad=True) for k, v in P.unpack(params).items()}
    opt = torch.optim.Adam(list(t.values()), lr=lr, betas=(b1, b2), eps=eps)
    xt, yt = torch.tensor(x), torch.tensor(y)
    want_losses = []
    for idx in batches:
        opt.zero_grad()
        h1 = torch.relu(xt[idx] @ t["W1"] + t["b1"])
        h2 = torch.relu(h1 @ t["W2"] + t["b2"])
        z3 = h2 @ t["w3"] + t["b3"][0]
        lt = torch.nn.functional.binary_cross_entropy_with_logits(z3, yt[idx])
        lt.backward()
        want_losses.append(lt.item())
        opt.step()
    want = P.pack({k: v.detach().numpy() for k, v in t.items()})
    np.testing.assert_allclose(losses, want_losses, rtol=1e-12)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-12)


def test_features_by_hand():
    x = P.features([3], [2], [0], [5], 11, [[0, 1, 0, 0, 0, 0, 0, 3]])
    want = [np.log(4), np.log(3), 0.0, 0.5, 0.0, np.log(2), 0, 0, 0, 0, 0, np.log(4)]
    np.testing.assert_allclose(x[0], want)
    assert P.features([3], [2], [0], [0], 1, [[0] * 8])[0, 3] == 0.0  # a single source


def test_schedule_by_enumeration():
    ids = np.arange(40)
    low = (ids % 3) == 0
    for run in range(8):
        got = P.tested(ids, low, run)
        for i in ids:
            assert got[i] == ((not low[i]) or ((run + i) % 4 == 0))
    # over any 4 consecutive runs a low clause is tested exactly once
    counts = sum(P.tested(ids, low, r).astype(int) for r in range(5, 9))
    assert (counts[low] == 1).all() and (counts[~low] == 4).all()


def test_hit_counts():
    dense = np.array([[0, 1], [2**64 - 1, 3], [0, 0]], dtype=np.uint64)
    np.testing.assert_array_equal(P.hit_counts(dense), [1, 66, 0])


def test_activity_closed_forms():
    decay = 0.95
    runs = 6
    always = np.ones((runs, 1))
    # geometric series: sum over r of decay**-r
    want = (decay ** -runs - 1) / (decay ** -1 - 1)
    assert abs(P.activity(always, decay)[0] - want) < 1e-12
    # a single hit in run r is worth decay**-r; later hits weigh more
    one = np.zeros((runs, runs))
    one[np.arange(runs), np.arange(runs)] = 3
    np.testing.assert_allclose(P.activity(one, decay), decay ** -np.arange(runs))
    # decay 1: activity counts the runs with a hit
    h = np.random.default_rng(1).integers(0, 3, (9, 50))
    np.testing.assert_array_equal(P.activity(h, 1.0), (h > 0).sum(axis=0))


def test_reduce_keep_by_enumeration():
    act = np.array([0.5, 2.0, 0.5, 1.0, 0.0, 2.0])
    ids = np.array([10, 11, 12, 13, 14, 15])
    assert list(P.reduce_keep(act, ids, 6)) == [10, 11, 12, 13, 14, 15]
    assert list(P.reduce_keep(act, ids, 3)) == [11, 13, 15]
    # 0.5 tie: the newer of 10 and 12 stays
    assert list(P.reduce_keep(act, ids, 4)) == [11, 12, 13, 15]
    assert list(P.reduce_keep(act, ids, 0)) == []
