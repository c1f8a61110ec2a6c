"""The fully connected corrective-forcing network (Sec. 2.1 and 2.2) and its
training: mean-square-error loss (Sec. 3.2, Table 1) minimised with Adam.

Test infrastructure only (see ``oracle/__init__``).

One network, shared by every element (Sec. 2.2), maps the element's
normalised nodal state to its normalised forcing:
    h_0 = xhat,  h_l = act(W_l h_{l-1} + b_l) for hidden layers,  yhat = W_L h_{L-1} + b_L,
with a linear output layer.  The paper's hidden activation is relu; the
workload measured here uses tanh.  Everything is float64; the weights the
network is given are first rounded to bfloat16 (``bf16_round``) so that the
oracle evaluates the same weights the device network stores.

Training minimises L = mean over the batch and the outputs of (yhat - y)^2
(the loss the paper reports is a mean square error).  The gradient is the
plain chain rule; Adam is Kingma and Ba's update with bias correction,
theta <- theta - lr mhat / (sqrt(vhat) + eps).
"""
import numpy as np


def bf16_round(x):
    """Round float32 values to the nearest bfloat16, ties to even; returns float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = x32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    isnan = np.isnan(x32)
    rounded = np.where(isnan, (bits.astype(np.uint32) | np.uint32(0x00400000)) & np.uint32(0xFFFF0000), rounded)
    return rounded.view(np.float32).astype(np.float64).reshape(x32.shape)


def activation(z, kind):
    if kind == "tanh":
        return np.tanh(z)
    if kind == "relu":
        return np.maximum(z, 0.0)
    raise ValueError(kind)


def activation_grad_from_output(h, kind):
    """d act / d z expressed through h = act(z)."""
    if kind == "tanh":
        return 1.0 - h * h
    if kind == "relu":
        return (h > 0.0).astype(np.float64)
    raise ValueError(kind)


def forward(params, x, act="tanh", quantise=False):
    """All layer outputs [h_0 = x, h_1, ..., yhat] for a batch x[B, n_in].
    ``params`` is a list of (W[out, in], b[out]).  quantise=True stores the
    input and every hidden layer's output as bfloat16 (the device network's
    precision for the activations between layers); the arithmetic stays float64."""
    h = np.asarray(x, dtype=np.float64)
    if quantise:
        h = bf16_round(h)
    outs = [h]
    L = len(params)
    for l, (W, b) in enumerate(params):
        z = h @ np.asarray(W, dtype=np.float64).T + np.asarray(b, dtype=np.float64)
        if l == L - 1:
            h = z
        else:
            h = activation(z, act)
            if quantise:
                h = bf16_round(h)
        outs.append(h)
    return outs


def mse_loss_and_grads(params, x, y, act="tanh", quantise=False):
    """Loss and its gradients [(dW, db), ...] for one batch (quantise: as in
    ``forward``; the backward pass is float64 either way)."""
    outs = forward(params, x, act, quantise)
    yhat = outs[-1]
    B, n_out = yhat.shape
    diff = yhat - y
    loss = float(np.mean(diff * diff))
    dz = 2.0 * diff / (B * n_out)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W = np.asarray(params[l][0], dtype=np.float64)
        grads[l] = (dz.T @ outs[l], dz.sum(axis=0))
        if l > 0:
            dz = (dz @ W) * activation_grad_from_output(outs[l], act)
    return loss, grads


def adam_update(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-7):
    """One Adam step (t counts from 1).  All lists hold (W, b) pairs; returns new lists."""
    new_p, new_m, new_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        pair_p, pair_m, pair_v = [], [], []
        for th, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = beta1 * mm + (1.0 - beta1) * g
            vv = beta2 * vv + (1.0 - beta2) * g * g
            mhat = mm / (1.0 - beta1 ** t)
            vhat = vv / (1.0 - beta2 ** t)
            pair_p.append(th - lr * mhat / (np.sqrt(vhat) + eps))
            pair_m.append(mm)
            pair_v.append(vv)
        new_p.append(tuple(pair_p))
        new_m.append(tuple(pair_m))
        new_v.append(tuple(pair_v))
    return new_p, new_m, new_v


def zeros_like_params(params):
    return [(np.zeros_like(np.asarray(W, dtype=np.float64)), np.zeros_like(np.asarray(b, dtype=np.float64)))
            for W, b in params]
