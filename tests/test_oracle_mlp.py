"""Pins of the FP64 surrogate-MLP reference against PyTorch's own GELU,
autograd and Adam (independent implementations), and finite differences."""
import numpy as np
import torch

from oracle import mlp as M


def _params(seed=0, scale=0.2):
    rng = np.random.default_rng(seed)
    return {n: rng.normal(0, scale, M.SHAPES[n]) for n in M.NAMES}


def test_gelu_matches_torch():
    x = np.linspace(-6, 6, 241)
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    y = torch.nn.functional.gelu(xt, approximate="tanh")
    assert np.max(np.abs(M.gelu(x) - y.detach().numpy())) < 1e-14
    y.sum().backward()
    assert np.max(np.abs(M.gelu_grad(x) - xt.grad.numpy())) < 1e-13


def test_grads_match_autograd():
    rng = np.random.default_rng(1)
    p = _params(1)
    X = rng.normal(0, 1, (37, M.N_IN))
    T = rng.normal(0, 1, (37, M.N_OUT))
    loss, g = M.loss_and_grads(p, X, T)
    tp = {n: torch.tensor(v, requires_grad=True) for n, v in p.items()}
    Xt, Tt = torch.tensor(X), torch.tensor(T)
    h = torch.nn.functional.gelu(Xt @ tp["W1"] + tp["b1"], approximate="tanh")
    h = torch.nn.functional.gelu(h @ tp["W2"] + tp["b2"], approximate="tanh")
    y = h @ tp["W3"] + tp["b3"]
    lt = torch.nn.functional.mse_loss(y, Tt)
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12
    for n in M.NAMES:
        assert np.max(np.abs(g[n] - tp[n].grad.numpy())) < 1e-12, n


def test_grads_central_difference():
    rng = np.random.default_rng(2)
    p = _params(2)
    X = rng.normal(0, 1, (5, M.N_IN))
    T = rng.normal(0, 1, (5, M.N_OUT))
    _, g = M.loss_and_grads(p, X, T)
    h = 1e-6
    for n in M.NAMES:
        flat = p[n].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            q = {k: v.copy() for k, v in p.items()}
            q[n].reshape(-1)[idx] += h
            lp, _ = M.loss_and_grads(q, X, T)
            q[n].reshape(-1)[idx] -= 2 * h
            lm, _ = M.loss_and_grads(q, X, T)
            assert abs((lp - lm) / (2 * h) - g[n].reshape(-1)[idx]) < 1e-7


def test_adam_matches_torch():
    rng = np.random.default_rng(3)
    p = _params(3)
    m = {n: np.zeros(M.SHAPES[n]) for n in M.NAMES}
    v = {n: np.zeros(M.SHAPES[n]) for n in M.NAMES}
    tp = [torch.tensor(p[n], requires_grad=True) for n in M.NAMES]
    opt = torch.optim.Adam(tp, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for k in (1, 2, 3):
        g = {n: rng.normal(0, 1, M.SHAPES[n]) for n in M.NAMES}
        p, m, v = M.adam_step(p, g, m, v, k, lr=1e-3)
        for t, n in zip(tp, M.NAMES):
            t.grad = torch.tensor(g[n])
        opt.step()
        for t, n in zip(tp, M.NAMES):
            assert np.max(np.abs(t.detach().numpy() - p[n])) < 1e-14


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 1000), [0.0, -0.0, 1.0, -3.5]])
    # values exactly halfway between two bfloat16 numbers (ties to even)
    base = rng.normal(0, 1, 200).astype(np.float32).view(np.uint32) & 0xFFFF0000
    x = np.concatenate([x, (base | 0x8000).view(np.float32).astype(np.float64)])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.round_bf16(x), want)


def test_rounded_grads_stay_near_exact():
    """With the BF16 rounding points the gradients move by about the BF16
    resolution (2^-8 relative), not more."""
    rng = np.random.default_rng(5)
    p = _params(5)
    X = M.round_bf16(rng.normal(0, 1, (64, M.N_IN)))
    T = rng.normal(0, 1, (64, M.N_OUT))
    _, g = M.loss_and_grads(p, X, T)
    _, gq = M.loss_and_grads(p, X, T, q=M.round_bf16)
    for n in M.NAMES:
        rel = np.linalg.norm(gq[n] - g[n]) / np.linalg.norm(g[n])
        assert 0 < rel < 1e-2, (n, rel)
