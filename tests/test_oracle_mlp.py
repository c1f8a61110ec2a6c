"""Pins of the oracle's forcing network, its training gradient and Adam
(Sec. 2.1, 2.2, Table 1), and of the forcing target of Eq. (5)."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import dg, forcing, mlp, projection
from oracle.basis import Basis


def _tiny(seed=0, dims=(8, 6, 6, 6, 8)):
    params = [(W.astype(np.float64), b.astype(np.float64) + 0.1) for W, b in synthetic.mlp_init(dims, seed)]
    rng = np.random.default_rng(seed + 1)
    x = rng.standard_normal((5, dims[0]))
    y = rng.standard_normal((5, dims[-1]))
    return params, x, y


def _torch_net(params, act):
    layers = []
    for l, (W, b) in enumerate(params):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(np.array(W)))
            lin.bias.copy_(torch.from_numpy(np.array(b)))
        layers.append(lin)
        if l < len(params) - 1:
            layers.append(torch.nn.Tanh() if act == "tanh" else torch.nn.ReLU())
    return torch.nn.Sequential(*layers)


@pytest.mark.parametrize("act", ["tanh", "relu"])
def test_forward_matches_torch(act):
    params, x, _ = _tiny()
    net = _torch_net(params, act)
    ref = net(torch.from_numpy(x)).detach().numpy()
    assert np.max(np.abs(mlp.forward(params, x, act)[-1] - ref)) < 1e-14


def test_gradients_match_finite_differences():
    params, x, y = _tiny(3)
    _, grads = mlp.mse_loss_and_grads(params, x, y)
    eps = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            flat = arr.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[idx]
                flat[idx] = old + eps
                lp, _ = mlp.mse_loss_and_grads(params, x, y)
                flat[idx] = old - eps
                lm, _ = mlp.mse_loss_and_grads(params, x, y)
                flat[idx] = old
                assert abs((lp - lm) / (2 * eps) - g.reshape(-1)[idx]) < 1e-7


@pytest.mark.parametrize("act", ["tanh", "relu"])
def test_gradients_match_autograd(act):
    params, x, y = _tiny(4)
    loss, grads = mlp.mse_loss_and_grads(params, x, y, act)
    net = _torch_net(params, act)
    out = net(torch.from_numpy(x))
    tl = torch.mean((out - torch.from_numpy(y)) ** 2)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-14
    lins = [m for m in net if isinstance(m, torch.nn.Linear)]
    for (gW, gb), lin in zip(grads, lins):
        assert np.max(np.abs(gW - lin.weight.grad.numpy())) < 1e-13
        assert np.max(np.abs(gb - lin.bias.grad.numpy())) < 1e-13


def test_adam_matches_torch_and_first_step_closed_form():
    params, x, y = _tiny(5)
    lr, eps = 1e-3, 1e-7
    net = _torch_net(params, "tanh")
    opt = torch.optim.Adam(net.parameters(), lr=lr, betas=(0.9, 0.999), eps=eps)
    m = mlp.zeros_like_params(params)
    v = mlp.zeros_like_params(params)
    p = params
    for t in range(1, 4):
        _, grads = mlp.mse_loss_and_grads(p, x, y)
        if t == 1:
            p1, _, _ = mlp.adam_update(p, grads, m, v, t, lr=lr, eps=eps)
            for (W1, b1), (W0, b0), (gW, gb) in zip(p1, p, grads):
                assert np.max(np.abs((W1 - W0) + lr * gW / (np.abs(gW) + eps))) < 1e-15
        p, m, v = mlp.adam_update(p, grads, m, v, t, lr=lr, eps=eps)
        opt.zero_grad()
        torch.mean((net(torch.from_numpy(x)) - torch.from_numpy(y)) ** 2).backward()
        opt.step()
    lins = [mm for mm in net if isinstance(mm, torch.nn.Linear)]
    for (W, b), lin in zip(p, lins):
        assert np.max(np.abs(W - lin.weight.detach().numpy())) < 1e-13
        assert np.max(np.abs(b - lin.bias.detach().numpy())) < 1e-13


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(7)
    np.seterr(under="ignore", over="ignore")
    vals = np.concatenate([
        rng.standard_normal(10000).astype(np.float32),
        (rng.standard_normal(1000) * 1e-38).astype(np.float32),          # subnormals
        np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 3.4e38, -3.4e38, 1e-45], dtype=np.float32),
        # exact ties: lower 16 bits 0x8000, with even and odd kept bit
        np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x3F80FFFF, 0x3F807FFF], dtype=np.uint32).view(np.float32),
    ])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    got = mlp.bf16_round(vals)
    assert np.array_equal(got, ref) or np.all((got == ref) | (np.isnan(got) & np.isnan(ref)))


def test_network_forcing_layout_and_mask():
    """Per-element rows are variable-major; the mask zeroes whole variables."""
    rng = np.random.default_rng(8)
    q = rng.standard_normal((5, 3, 8))
    params = [(np.eye(40), np.zeros(40))]
    norm = forcing.Normalisation(np.zeros(5), np.ones(5), np.zeros(5), np.ones(5), mask=(0, 1, 1, 1, 0))
    s = forcing.network_forcing(q, params, norm)
    assert np.array_equal(s[1:4], q[1:4]) and np.all(s[[0, 4]] == 0)
    X = forcing.element_rows(q)
    assert X[2, 1 * 8 + 5] == q[1, 2, 5]


def test_forcing_target_vanishes_for_equal_orders():
    prm = dg.Params(N=2, P=3, Re=200.0)
    q = dg.to_blocks(synthetic.random_state(2, 3, seed=9), 2, 3)
    x, y = forcing.forcing_target(q, prm, prm)
    assert np.max(np.abs(y)) < 1e-12 * np.max(np.abs(dg.residual(q, prm)))


def test_forcing_target_is_conservative():
    """Both residuals conserve and G keeps element integrals, so each variable's
    integral of the target vanishes."""
    prm_hi = dg.Params(N=2, P=6, Re=1600.0, Cs=0.1)
    prm_lo = dg.Params(N=2, P=3, Re=1600.0)
    q = dg.tgv_initial_condition(prm_hi)
    x, y = forcing.forcing_target(q, prm_hi, prm_lo)
    yf = forcing.rows_to_field(y, 5, 64)
    yb = dg.to_blocks(yf, 2, 3)
    Wq = dg.quadrature_weights(Basis(3)) * prm_lo.J
    R_hi = dg.residual(q, prm_hi)
    for v in range(5):
        scale = np.sum(dg.quadrature_weights(Basis(6)) * prm_hi.J * np.abs(R_hi[v]))
        assert abs(np.sum(Wq * yb[v])) < 1e-13 * max(scale, 1.0)
    assert np.max(np.abs(dg.to_blocks(forcing.rows_to_field(x, 5, 64), 2, 3) - projection.project(q, 6, 3))) == 0


def test_quantised_forward_stores_bf16_and_is_exact_on_representable_values():
    """quantise=True rounds the input and the hidden outputs to bfloat16: every
    stored activation is a bfloat16 value, and a network whose activations are
    small integers (exact in bfloat16) gives the unquantised result."""
    rng = np.random.default_rng(13)
    params, x, _ = _tiny(6)
    outs = mlp.forward(params, x, "tanh", quantise=True)
    for h in outs[:-1]:
        assert np.array_equal(mlp.bf16_round(h), h)
    # integer weights, integer inputs, relu: activations stay small integers
    dims = (6, 5, 4, 3)
    ip = [(rng.integers(-2, 3, size=(dims[l + 1], dims[l])).astype(np.float64),
           rng.integers(-2, 3, size=dims[l + 1]).astype(np.float64)) for l in range(3)]
    xi = rng.integers(-3, 4, size=(7, 6)).astype(np.float64)
    a = mlp.forward(ip, xi, "relu", quantise=True)
    b = mlp.forward(ip, xi, "relu")
    assert all(np.array_equal(u, v) for u, v in zip(a, b))
    la, ga = mlp.mse_loss_and_grads(ip, xi, np.zeros((7, 3)), "relu", quantise=True)
    lb, gb = mlp.mse_loss_and_grads(ip, xi, np.zeros((7, 3)), "relu")
    assert la == lb and all(np.array_equal(p[0], q[0]) and np.array_equal(p[1], q[1]) for p, q in zip(ga, gb))
