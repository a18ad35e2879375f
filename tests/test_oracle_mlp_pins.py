"""Pins for the FP64 reference of the candidate-scoring network (CPU only).

The reference in oracle/mlp.c is tied to computations it does not share:
finite differences of its own loss, an independent float64 autograd
implementation (torch on the CPU), torch's Adam in float64, torch's
float32 -> bfloat16 conversion, and node features worked out by hand.
"""
import numpy as np
import pytest
import torch

import oracle

NP = 4609
H, IN = 64, 5


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, NP)


def _split(p):
    o = 0
    W1 = p[o:o + H * IN].reshape(H, IN); o += H * IN
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def _torch_loss(p, x, t):
    W1, b1, W2, b2, w3, b3 = _split(p)
    h1 = torch.relu(x @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    y = h2 @ w3 + b3
    return ((y - t) ** 2).sum() / (2 * len(t)), y


def test_parameter_count():
    assert oracle.mlp_nparams() == NP == H * IN + H + H * H + H + H + 1


def test_bf16_round_matches_torch_and_ties():
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 2000),
                        rng.normal(0, 1e4, 2000)]).astype(np.float32)
    # exact ties between two bfloat16 neighbours: 1 + 2^-8 (to even: 1.0),
    # 1 + 3 * 2^-8 (to even: 1 + 2^-6), and their negatives
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), -(1 + 3 * 2.0 ** -8)],
                    dtype=np.float32)
    a = np.concatenate([a, ties, np.array([0.0, -0.0, 1.0, 2.0 ** -100], np.float32)])
    got = oracle.bf16_round(a)
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert got[-8] == 1.0 and got[-7] == np.float32(1 + 2.0 ** -6)


def test_forward_and_gradient_match_float64_autograd():
    p = _params(2)
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1.5, (300, IN))
    t = rng.normal(0, 1, 300)
    loss, g = oracle.mlp_loss_grad(p, x, t)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    lt, yt = _torch_loss(pt, torch.tensor(x), torch.tensor(t))
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-12 * max(1.0, abs(loss))
    np.testing.assert_allclose(oracle.mlp_forward(p, x), yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_gradient_finite_differences():
    p = _params(4)
    rng = np.random.default_rng(5)
    x = rng.normal(0, 1.5, (64, IN))
    t = rng.normal(0, 1, 64)
    _, g = oracle.mlp_loss_grad(p, x, t)
    # every parameter block, including the biases and the output bias
    idx = np.concatenate([rng.choice(H * IN, 40, replace=False),
                          H * IN + rng.choice(H, 10, replace=False),
                          H * IN + H + rng.choice(H * H, 60, replace=False),
                          H * IN + H + H * H + rng.choice(H, 10, replace=False),
                          H * IN + 2 * H + H * H + rng.choice(H, 10, replace=False),
                          [NP - 1]])
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (oracle.mlp_loss_grad(pp, x, t)[0] - oracle.mlp_loss_grad(pm, x, t)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_linear_special_case_closed_form():
    # With every hidden unit active and W2 = I, the network is affine:
    # y = w3 . (W1 x + b1 + b2) + b3.
    rng = np.random.default_rng(6)
    p = np.zeros(NP)
    W1 = rng.normal(0, 0.1, (H, IN))
    b1 = np.full(H, 10.0)      # keeps the first layer positive for |x| < 5
    w3 = rng.normal(0, 1, H)
    o = 0
    p[o:o + H * IN] = W1.ravel(); o += H * IN
    p[o:o + H] = b1; o += H
    p[o:o + H * H] = np.eye(H).ravel(); o += H * H
    p[o:o + H] = 0.5; o += H
    p[o:o + H] = w3; o += H
    p[o] = -2.0
    x = rng.uniform(-4, 4, (50, IN))
    want = (x @ W1.T + b1 + 0.5) @ w3 - 2.0
    np.testing.assert_allclose(oracle.mlp_forward(p, x), want, rtol=1e-12)


def test_adam_matches_torch_float64():
    rng = np.random.default_rng(7)
    theta0 = rng.normal(0, 1, 200)
    grads = [rng.normal(0, 1, 200) for _ in range(4)]
    th, m, v = theta0.copy(), np.zeros(200), np.zeros(200)
    for step, g in enumerate(grads, start=1):
        oracle.adam_step(th, m, v, g, 1e-2, 0.9, 0.999, 1e-8, step)
    pt = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for g in grads:
        opt.zero_grad()
        pt.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(th, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_node_features_by_hand():
    # 0 -> 1 (p .5), 0 -> 2 (p .25), 1 -> 2 (p 1), 2 -> 0 (p .125), 3 isolated
    row_ptr = np.array([0, 2, 3, 4, 4], np.uint64)
    col = np.array([1, 2, 2, 0], np.uint32)
    prob = np.array([0.5, 0.25, 1.0, 0.125], np.float32)
    f = oracle.node_features(row_ptr, col, prob)
    indeg = [1, 1, 2, 0]
    outdeg = [2, 1, 1, 0]
    psum = [0.75, 1.0, 0.125, 0.0]
    two = [1 + 1, 1, 2, 0]
    want = np.log1p(np.array([indeg, outdeg, psum, two], np.float64).T)
    np.testing.assert_allclose(f, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("bad", ["w2_transposed", "relu_dropped"])
def test_planted_mistakes_fail_the_pins(bad):
    # The autograd pin must catch a transposed hidden layer or a missing
    # ReLU: build the wrong model in torch and check it disagrees with the
    # oracle on the same inputs.
    p = _params(8)
    rng = np.random.default_rng(9)
    x = torch.tensor(rng.normal(0, 1.5, (100, IN)))
    W1, b1, W2, b2, w3, b3 = (torch.tensor(np.asarray(a)) for a in _split(p))
    h1 = torch.relu(x @ W1.T + b1)
    if bad == "w2_transposed":
        y = torch.relu(h1 @ W2 + b2) @ w3 + b3
    else:
        y = (h1 @ W2.T + b2) @ w3 + b3
    assert not np.allclose(oracle.mlp_forward(p, x.numpy()), y.numpy(), rtol=1e-6)
