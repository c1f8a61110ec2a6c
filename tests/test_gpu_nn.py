"""GPU parity of the forcing network (Sec. 2.2, Eq. (4)) and its training
(MSE loss, Adam) against the CPU oracle, through the C ABI.

Tolerances: the network runs on bf16 matrix cores with float32 accumulation,
so the forcing matches the float64 oracle (same bf16 weights) to 1e-2
relative (L2 over the field), gradients to 1e-2 relative per tensor, and the
kinetic-energy history of a corrected run to 1e-3 relative.  Weight rounding
to bf16 is bitwise.
"""
import numpy as np
import pytest

import synthetic
from helpers import rel_l2, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DIMS = [320, 256, 256, 256, 320]
# physical-scale normalisation of the randomly initialised network:
# mu_in, sigma_in, mu_out, sigma_out per conserved variable
NORM = [1.0, 0.0, 0.0, 0.0, synthetic.TGV_ENERGY_LEVEL,
        0.01, 1.0, 1.0, 1.0, 1.0,
        0.0, 0.0, 0.0, 0.0, 0.0,
        1e-3, 1e-3, 1e-3, 1e-3, 1e-3]


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_11571_amd import binding
    binding.lib()
    return binding


def _oracle_model(layers, norm=NORM, mask=(1, 1, 1, 1, 1)):
    from oracle import forcing, mlp
    params = [(mlp.bf16_round(W), b.astype(np.float64)) for W, b in layers]
    n = forcing.Normalisation(norm[0:5], norm[5:10], norm[10:15], norm[15:20], mask)
    return params, n


def _to_gpu(a, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def test_bf16_weight_copies_bitwise(B):
    from oracle import mlp
    say("bf16 copies")
    layers = synthetic.mlp_init(DIMS, seed=0)
    model = B.Model(DIMS, B.pack_params(layers), NORM)
    torch.cuda.synchronize()
    wbf = model.wbf.cpu().numpy().view(np.uint16)

    def unfragment(flat, rows, cols):
        # the copies are in the matrix cores' fragment order: element [n][k]
        # of a [rows][cols] matrix sits in the 1 KB block of (n // 16, k // 32)
        # at lane n % 16 + 16 ((k % 32) // 8), entry k % 8
        n, k = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
        idx = (((n // 16) * (cols // 32) + k // 32) * 64 + n % 16 + 16 * ((k % 32) // 8)) * 8 + k % 8
        return flat[idx]

    off = 0
    for W, _ in layers:
        out_d, in_d = W.shape
        pin, pout = (in_d + 31) // 32 * 32, (out_d + 31) // 32 * 32
        Wb = unfragment(wbf[off:off + pout * pin], pout, pin)
        off += pout * pin
        WTb = unfragment(wbf[off:off + pout * pin], pin, pout)
        off += pout * pin
        ref = (mlp.bf16_round(W).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
        assert np.array_equal(Wb[:out_d, :in_d], ref)
        assert np.array_equal(WTb[:in_d, :out_d], ref.T)
        assert not Wb[out_d:].any() and not Wb[:, in_d:].any()


@pytest.mark.parametrize("N", [16, 3])
def test_forcing_matches_oracle(B, N):
    """C3 network (320 -> 256 x 3 tanh -> 320, Gaussian init, seed 0) on a
    perturbed TGV state; N = 3 leaves a ragged last block of rows."""
    from oracle import dg, forcing
    say("forcing", N)
    layers = synthetic.mlp_init(DIMS, seed=0)
    params, norm = _oracle_model(layers)
    prm = dg.Params(N=N, P=3, Re=200.0)
    q = dg.tgv_initial_condition(prm).copy()
    q[1:4] += 0.05 * np.random.default_rng(1).standard_normal(q[1:4].shape)
    qf = dg.to_flat(q)
    ref = forcing.network_forcing(qf, params, norm)
    m = B.Mesh(N, 3, 200.0)
    model = B.Model(DIMS, B.pack_params(layers), NORM, train=False)
    out = m.field(0.0)
    B.nn_forcing(model, m, _to_gpu(qf), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    err = rel_l2(got, ref)
    print("forcing rel L2", err)
    assert err < 1e-2
    # accumulation: a second call adds the same forcing again
    B.nn_forcing(model, m, _to_gpu(qf), out)
    assert rel_l2(out.cpu().numpy(), 2 * got) < 1e-15


def test_corrected_ke_history(B):
    """P = 3 TGV at Re 200 on 4^3 elements with the network at every stage:
    kinetic energy over 100 steps matches the oracle to 1e-3."""
    from oracle import dg, forcing, rk
    say("corrected KE history")
    N, P, Re = 4, 3, 200.0
    layers = synthetic.mlp_init(DIMS, seed=0)
    params, norm = _oracle_model(layers)
    prm = dg.Params(N=N, P=P, Re=Re)
    q0 = dg.tgv_initial_condition(prm)
    dt = dg.stable_dt(q0, prm)
    ke_ref = []
    rk.integrate(q0, dt, 100, lambda qq, t: forcing.corrected_rhs(qq, prm, params, norm),
                 callback=lambda n, qq: ke_ref.append(dg.kinetic_energy(qq, prm)))
    m = B.Mesh(N, P, Re)
    model = B.Model(DIMS, B.pack_params(layers), NORM, train=False)
    q = _to_gpu(dg.to_flat(q0))
    k = m.field(0.0)
    ke = []
    for n in range(100):
        B.dg_rk_step(m, q, k, dt, 1, model=model)
        ke.append(B.dg_diagnostics(m, q)[0].item())
    ke, ke_ref = np.array(ke), np.array(ke_ref)
    err = np.max(np.abs(ke - ke_ref) / ke_ref)
    print("KE history max rel", err)
    assert err < 1e-3
    # the network changes the solution: the uncorrected run differs
    q2 = _to_gpu(dg.to_flat(q0))
    B.dg_rk_step(m, q2, k, dt, 100)
    assert abs(B.dg_diagnostics(m, q2)[0].item() - ke[-1]) > 10 * err * ke[-1]


@pytest.mark.parametrize("batch", [256, 200])
def test_train_step_gradients_and_adam(B, batch):
    from oracle import mlp
    say("train step", batch)
    dims = DIMS
    layers = synthetic.mlp_init(dims, seed=0)
    layers = [(W, b + 0.01) for W, b in layers]
    rng = np.random.default_rng(2)
    x = np.empty((batch, 320), dtype=np.float32)
    x[:, :64] = 1.0 + 0.01 * rng.standard_normal((batch, 64))
    x[:, 64:256] = rng.standard_normal((batch, 192))
    x[:, 256:] = synthetic.TGV_ENERGY_LEVEL + rng.standard_normal((batch, 64))
    y = (1e-3 * rng.standard_normal((batch, 320))).astype(np.float32)
    model = B.Model(dims, B.pack_params(layers), NORM)
    p_before = model.params.cpu().numpy().astype(np.float64)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    B.nn_train_step(model, _to_gpu(x, np.float32), _to_gpu(y, np.float32), lr=1e-3, loss=loss)
    torch.cuda.synchronize()
    # oracle gradient at the same (bf16-rounded) weights, on normalised data
    params, norm = _oracle_model(layers)
    n_p = 64
    xh = (x.astype(np.float64) - np.repeat(norm.mu_in, n_p)) / np.repeat(norm.sigma_in, n_p)
    yt = (y.astype(np.float64) - np.repeat(norm.mu_out, n_p)) / np.repeat(norm.sigma_out, n_p)
    loss_ref, grads = mlp.mse_loss_and_grads(params, xh, yt)
    assert abs(loss.item() / loss_ref - 1) < 1e-2
    g_gpu = B.unpack_params(model.grad.cpu().numpy().astype(np.float64), dims)
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(g_gpu, grads)):
        eW, eb = rel_l2(gW, rW), rel_l2(gb, rb)
        print("layer", l, "grad rel L2", eW, eb)
        assert eW < 1e-2 and eb < 1e-2
    # Adam step 1 on the device's own gradient, float64 reference
    g_flat = model.grad.cpu().numpy().astype(np.float64)
    m1 = 0.1 * g_flat
    v1 = 0.001 * g_flat * g_flat
    ref = p_before - 1e-3 * (m1 / 0.1) / (np.sqrt(v1 / 0.001) + 1e-7)
    assert np.max(np.abs(model.params.cpu().numpy() - ref)) < 1e-6 * np.max(np.abs(ref))


def test_training_reduces_loss(B):
    say("training loop")
    dims = DIMS
    layers = synthetic.mlp_init(dims, seed=0)
    rng = np.random.default_rng(4)
    x = np.empty((512, 320), dtype=np.float32)
    x[:, :64] = 1.0 + 0.01 * rng.standard_normal((512, 64))
    x[:, 64:256] = rng.standard_normal((512, 192))
    x[:, 256:] = synthetic.TGV_ENERGY_LEVEL + rng.standard_normal((512, 64))
    y = (1e-3 * np.tanh(x[:, 64:256].sum(axis=1, keepdims=True) / 10) * np.ones((1, 320))).astype(np.float32)
    model = B.Model(dims, B.pack_params(layers), NORM)
    xg, yg = _to_gpu(x, np.float32), _to_gpu(y, np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    for it in range(60):
        B.nn_train_step(model, xg, yg, lr=1e-3, loss=loss)
        losses.append(loss.item())
    print("loss", losses[0], losses[-1])
    assert losses[-1] < 0.2 * losses[0]


def test_data_stats_match_oracle(B):
    """Per-variable normalisation of a training set (device reduction) vs the
    oracle's mean / standard deviation."""
    from oracle import forcing
    say("data stats")
    rng = np.random.default_rng(9)
    rows = 3000
    x = np.empty((rows, 320), dtype=np.float32)
    x[:, :64] = 1.0 + 0.02 * rng.standard_normal((rows, 64))
    x[:, 64:256] = rng.standard_normal((rows, 192))
    x[:, 256:] = synthetic.TGV_ENERGY_LEVEL + rng.standard_normal((rows, 64))
    y = (1e-2 * rng.standard_normal((rows, 320))).astype(np.float32)
    y[:, :64] = 0.0        # a constant variable: its sigma hits the floor
    got = np.array(B.nn_data_stats(_to_gpu(x, np.float32), _to_gpu(y, np.float32), 64))
    ref = forcing.normalisation_from_pairs(x, y).as_array()
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-10


def test_train_step_row_indices(B):
    """A step on rows idx of (x, y) equals a step on the gathered rows."""
    say("train idx")
    layers = synthetic.mlp_init(DIMS, seed=3)
    rng = np.random.default_rng(5)
    x = np.empty((600, 320), dtype=np.float32)
    x[:, :64] = 1.0
    x[:, 64:256] = rng.standard_normal((600, 192))
    x[:, 256:] = synthetic.TGV_ENERGY_LEVEL
    y = (1e-3 * rng.standard_normal((600, 320))).astype(np.float32)
    idx = rng.permutation(600)[:256].astype(np.int32)
    m1 = B.Model(DIMS, B.pack_params(layers), NORM)
    m2 = B.Model(DIMS, B.pack_params(layers), NORM)
    B.nn_train_step(m1, _to_gpu(x, np.float32), _to_gpu(y, np.float32), idx=torch.from_numpy(idx).cuda())
    B.nn_train_step(m2, _to_gpu(x[idx], np.float32), _to_gpu(y[idx], np.float32))
    torch.cuda.synchronize()
    assert torch.equal(m1.params, m2.params) and torch.equal(m1.grad, m2.grad)


def test_corrected_ke_history_C3(B):
    """The corrected run at its throughput size: 16^3 elements, P = 3, Re 200,
    the Gaussian network at every stage, 100 steps.  The kinetic energy after
    every step matches the oracle's history (tests/golden/c3_ke_history.json,
    written by the committed oracle-only script beside it) to 1e-3."""
    import json
    import os
    from oracle import dg
    say("corrected KE history C3 16^3")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c3_ke_history.json")))
    assert gold["dims"] == DIMS and gold["norm"] == NORM
    N, P, Re = gold["N"], gold["P"], gold["Re"]
    m = B.Mesh(N, P, Re)
    q = m.field()
    B.dg_init_tgv(m, q)
    dt = B.dg_stable_dt(m, q)
    assert abs(dt / gold["dt"] - 1) < 1e-13
    model = B.Model(DIMS, B.pack_params(synthetic.mlp_init(DIMS, seed=gold["seed"])), NORM, train=False)
    k = m.field(0.0)
    ke = []
    for n in range(len(gold["ke"])):
        B.dg_rk_step(m, q, k, dt, 1, model=model)
        ke.append(B.dg_diagnostics(m, q)[0].item())
    ke, ke_ref = np.array(ke), np.array(gold["ke"])
    err = np.max(np.abs(ke - ke_ref) / ke_ref)
    print("C3 KE history max rel", err)
    assert err < 1e-3


def test_adam_several_steps(B):
    """Four Adam steps on fixed data: after each, the device's float32 master
    weights equal the float64 Adam recursion (Kingma-Ba with bias correction,
    beta = (0.9, 0.999), eps = 1e-7) driven by the device's own gradients,
    and the fourth step's gradient matches the oracle's at the device's
    current weights.  From step 2 on, swapped or mis-corrected moments change
    the update by ~1e-4 of a weight, far above the 1e-6 tolerance."""
    from oracle import mlp
    say("adam several steps")
    dims = DIMS
    layers = synthetic.mlp_init(dims, seed=1)
    layers = [(W, b + 0.01) for W, b in layers]
    rng = np.random.default_rng(12)
    batch = 256
    x = np.empty((batch, 320), dtype=np.float32)
    x[:, :64] = 1.0 + 0.01 * rng.standard_normal((batch, 64))
    x[:, 64:256] = rng.standard_normal((batch, 192))
    x[:, 256:] = synthetic.TGV_ENERGY_LEVEL + rng.standard_normal((batch, 64))
    y = (1e-3 * rng.standard_normal((batch, 320))).astype(np.float32)
    model = B.Model(dims, B.pack_params(layers), NORM)
    xg, yg = _to_gpu(x, np.float32), _to_gpu(y, np.float32)
    p_ref = B.unpack_params(model.params.cpu().numpy().astype(np.float64), dims)
    m_ref, v_ref = mlp.zeros_like_params(p_ref), mlp.zeros_like_params(p_ref)
    lr = 1e-3
    for t in range(1, 5):
        p_dev_before = B.unpack_params(model.params.cpu().numpy().astype(np.float64), dims)
        B.nn_train_step(model, xg, yg, lr=lr)
        torch.cuda.synchronize()
        g_dev = B.unpack_params(model.grad.cpu().numpy().astype(np.float64), dims)
        p_ref, m_ref, v_ref = mlp.adam_update(p_ref, g_dev, m_ref, v_ref, t, lr=lr)
        p_dev = B.unpack_params(model.params.cpu().numpy().astype(np.float64), dims)
        scale = max(np.max(np.abs(W)) for W, _ in p_ref)
        err = max(max(np.max(np.abs(a - b)) for a, b in zip(pd, pr)) for pd, pr in zip(p_dev, p_ref))
        moved = max(max(np.max(np.abs(a - b)) for a, b in zip(pd, pb)) for pd, pb in zip(p_dev, p_dev_before))
        print("adam step", t, "max |dev - ref|", err, "max update", moved)
        assert err < 1e-6 * scale, (t, err)
        assert moved > 100 * err
    # the last step's gradient at the weights the device used for it
    params, norm = _oracle_model(p_dev_before)
    n_p = 64
    xh = (x.astype(np.float64) - np.repeat(norm.mu_in, n_p)) / np.repeat(norm.sigma_in, n_p)
    yt = (y.astype(np.float64) - np.repeat(norm.mu_out, n_p)) / np.repeat(norm.sigma_out, n_p)
    _, grads = mlp.mse_loss_and_grads(params, xh, yt)
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(g_dev, grads)):
        assert rel_l2(gW, rW) < 1e-2 and rel_l2(gb, rb) < 1e-2, l


DIMS_P2 = [135, 256, 256, 256, 135]


def test_forcing_and_gradients_P2(B):
    """The network of the P_LO = 2 cases (Table 1, 1a - 2b): 135 -> 256 x 3
    tanh -> 135 (five variables x 27 nodes; the device pads 135 to 160).
    Forcing on a perturbed 4^3 Taylor-Green state and one training step's
    gradients against the oracle."""
    from oracle import dg, forcing, mlp
    say("P2 network forcing and gradients")
    layers = synthetic.mlp_init(DIMS_P2, seed=4)
    layers = [(W, b + 0.01) for W, b in layers]
    params, norm = _oracle_model(layers)
    prm = dg.Params(N=4, P=2, Re=30.0)
    q = dg.tgv_initial_condition(prm).copy()
    q[1:4] += 0.05 * np.random.default_rng(8).standard_normal(q[1:4].shape)
    qf = dg.to_flat(q)
    ref = forcing.network_forcing(qf, params, norm)
    m = B.Mesh(4, 2, 30.0)
    model = B.Model(DIMS_P2, B.pack_params(layers), NORM)
    out = m.field(0.0)
    B.nn_forcing(model, m, _to_gpu(qf), out)
    torch.cuda.synchronize()
    err = rel_l2(out.cpu().numpy(), ref)
    print("P2 forcing rel L2", err)
    assert err < 1e-2
    batch, n_p = 200, 27
    rng = np.random.default_rng(9)
    x = np.empty((batch, 135), dtype=np.float32)
    x[:, :27] = 1.0 + 0.01 * rng.standard_normal((batch, 27))
    x[:, 27:108] = rng.standard_normal((batch, 81))
    x[:, 108:] = synthetic.TGV_ENERGY_LEVEL + rng.standard_normal((batch, 27))
    y = (1e-3 * rng.standard_normal((batch, 135))).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    B.nn_train_step(model, _to_gpu(x, np.float32), _to_gpu(y, np.float32), lr=1e-3, loss=loss)
    torch.cuda.synchronize()
    xh = (x.astype(np.float64) - np.repeat(norm.mu_in, n_p)) / np.repeat(norm.sigma_in, n_p)
    yt = (y.astype(np.float64) - np.repeat(norm.mu_out, n_p)) / np.repeat(norm.sigma_out, n_p)
    loss_ref, grads = mlp.mse_loss_and_grads(params, xh, yt)
    assert abs(loss.item() / loss_ref - 1) < 1e-2
    g_gpu = B.unpack_params(model.grad.cpu().numpy().astype(np.float64), DIMS_P2)
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(g_gpu, grads)):
        eW, eb = rel_l2(gW, rW), rel_l2(gb, rb)
        print("P2 layer", l, "grad rel L2", eW, eb)
        assert eW < 1e-2 and eb < 1e-2


@pytest.mark.parametrize("dims", [[320, 96, 256, 160, 320], [320, 384, 320]])
def test_forcing_and_gradients_other_widths(B, dims):
    """Hidden widths other than 256 (P = 3, five variables in and out):
    96 -> 256 -> 160 leaves wavefronts without a column tile in one layer
    and with one in the next (forward and backward chains); 384 is wider
    than the 320 columns a wavefront keeps in registers, so those layers run
    the generic product.  Forcing on a perturbed 4^3 Taylor-Green state and
    one training step's loss and gradients against the oracle."""
    from oracle import dg, forcing, mlp
    say("network widths", dims)
    layers = synthetic.mlp_init(dims, seed=6)
    layers = [(W, b + 0.01) for W, b in layers]
    params, norm = _oracle_model(layers)
    prm = dg.Params(N=4, P=3, Re=200.0)
    q = dg.tgv_initial_condition(prm).copy()
    q[1:4] += 0.05 * np.random.default_rng(10).standard_normal(q[1:4].shape)
    qf = dg.to_flat(q)
    ref = forcing.network_forcing(qf, params, norm)
    m = B.Mesh(4, 3, 200.0)
    model = B.Model(dims, B.pack_params(layers), NORM)
    out = m.field(0.0)
    B.nn_forcing(model, m, _to_gpu(qf), out)
    torch.cuda.synchronize()
    err = rel_l2(out.cpu().numpy(), ref)
    print("forcing rel L2", err)
    assert err < 1e-2
    batch, n_p = 200, 64
    rng = np.random.default_rng(11)
    x = np.empty((batch, 320), dtype=np.float32)
    x[:, :64] = 1.0 + 0.01 * rng.standard_normal((batch, 64))
    x[:, 64:256] = rng.standard_normal((batch, 192))
    x[:, 256:] = synthetic.TGV_ENERGY_LEVEL + rng.standard_normal((batch, 64))
    y = (1e-3 * rng.standard_normal((batch, 320))).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    B.nn_train_step(model, _to_gpu(x, np.float32), _to_gpu(y, np.float32), lr=1e-3, loss=loss)
    torch.cuda.synchronize()
    xh = (x.astype(np.float64) - np.repeat(norm.mu_in, n_p)) / np.repeat(norm.sigma_in, n_p)
    yt = (y.astype(np.float64) - np.repeat(norm.mu_out, n_p)) / np.repeat(norm.sigma_out, n_p)
    loss_ref, grads = mlp.mse_loss_and_grads(params, xh, yt)
    assert abs(loss.item() / loss_ref - 1) < 1e-2
    g_gpu = B.unpack_params(model.grad.cpu().numpy().astype(np.float64), dims)
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(g_gpu, grads)):
        eW, eb = rel_l2(gW, rW), rel_l2(gb, rb)
        print("layer", l, "grad rel L2", eW, eb)
        assert eW < 1e-2 and eb < 1e-2
