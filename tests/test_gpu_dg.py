"""GPU parity of the FP64 DG path (libdgnn.so through its C ABI) against the
CPU oracle: initial condition, residual p(q) (Eq. (1)/(3)), Runge-Kutta steps,
diagnostics, filter G, forcing target (Eq. (5)), error norm (Eq. (9)).

Tolerance: the residual and states agree to 1e-12 relative (L2, per
variable) and 1e-11 relative in the infinity norm; both implementations are
float64 and differ only in summation order.
"""
import numpy as np
import pytest

import synthetic
from helpers import field_parity, periodic_patch, rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_11571_amd import binding
    binding.lib()
    return binding


def _oracle():
    from oracle import dg, forcing, projection, rk
    return dg, forcing, projection, rk


def _to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("N,P", [(4, 3), (3, 5), (2, 8)])
def test_tgv_initial_condition(B, N, P):
    dg, *_ = _oracle()
    say("tgv", N, P)
    m = B.Mesh(N, P, 30.0)
    q = m.field()
    B.dg_init_tgv(m, q)
    torch.cuda.synchronize()
    ref = dg.to_flat(dg.tgv_initial_condition(dg.Params(N=N, P=P, Re=30.0)))
    assert np.max(np.abs(q.cpu().numpy() - ref)) < 1e-13 * np.max(np.abs(ref))


def _residual_case(B, N, P, Re, Cs, viscous, q_flat):
    dg, *_ = _oracle()
    m = B.Mesh(N, P, Re, Cs=Cs, viscous=viscous)
    q = _to_gpu(q_flat)
    R = m.field(0.0)
    B.dg_residual(m, q, R)
    torch.cuda.synchronize()
    prm = dg.Params(N=N, P=P, Re=Re, Cs=Cs, viscous=viscous)
    ref = dg.to_flat(dg.residual(dg.to_blocks(q_flat, N, P), prm))
    return R.cpu().numpy(), ref


def test_residual_tgv_C1(B):
    """Re 30, Mach 0.1, 4^3 elements, P = 3, TGV initial state."""
    dg, *_ = _oracle()
    say("residual tgv C1")
    q = dg.to_flat(dg.tgv_initial_condition(dg.Params(N=4, P=3, Re=30.0)))
    got, ref = _residual_case(B, 4, 3, 30.0, 0.0, True, q)
    l2, li = field_parity(got, ref, 1e-12)
    print("C1 residual rel L2", l2, "rel inf", li)
    assert np.all(l2 < 1e-12) and np.all(li < 1e-11)


@pytest.mark.parametrize("N,P,Cs,viscous", [
    (3, 1, 0.0, True), (3, 2, 0.1, True), (3, 3, 0.0, False), (2, 4, 0.1, True),
    (3, 5, 0.0, True), (2, 6, 0.1, True), (2, 7, 0.0, True), (2, 8, 0.1, True), (1, 3, 0.0, True),
    # 343 elements at P = 8: more blocks than the GPU holds at once
    (7, 8, 0.1, True), (7, 8, 0.0, False)])
def test_residual_random_states(B, N, P, Cs, viscous):
    say("residual random", N, P, Cs, viscous)
    q = synthetic.random_state(N, P, seed=100 + 10 * N + P)
    got, ref = _residual_case(B, N, P, 200.0, Cs, viscous, q)
    l2, li = field_parity(got, ref, 1e-12)
    print("random residual rel L2", l2, "rel inf", li)
    assert np.all(l2 < 1e-12) and np.all(li < 1e-11)


@pytest.mark.parametrize("P,Cs", [(6, 0.0), (8, 0.0), (8, 0.1), (6, 0.1)])
def test_residual_full_size_sampled(B, P, Cs):
    """16^3 elements at Re 1600 (the throughput configuration): the residual of
    a perturbed TGV state on sampled elements, each checked against the oracle
    on the 5^3-element periodic patch around it (BR1 reaches two elements)."""
    dg, *_ = _oracle()
    N = 16
    say("residual full size", P, Cs)
    prm = dg.Params(N=N, P=P, Re=1600.0, Cs=Cs)
    q = dg.tgv_initial_condition(prm).copy()
    q[1:4] += 0.01 * np.random.default_rng(3).standard_normal(q[1:4].shape)
    q_flat = dg.to_flat(q)
    m = B.Mesh(N, P, 1600.0, Cs=Cs)
    qg = _to_gpu(q_flat)
    R = m.field(0.0)
    B.dg_residual(m, qg, R)
    torch.cuda.synchronize()
    Rb = dg.to_blocks(R.cpu().numpy(), N, P)
    for centre in [(0, 0, 0), (15, 7, 3), (8, 8, 8), (3, 15, 12)]:
        patch = periodic_patch(q, centre, 2)
        ref = dg.residual(patch, prm)[:, 2, 2, 2]
        got = Rb[:, centre[0], centre[1], centre[2]]
        l2, li = field_parity(got, ref, 1e-12)
        assert np.all(l2 < 1e-12) and np.all(li < 1e-11), (centre, l2, li)


def test_residual_C1_against_extended_precision(B):
    """The device residual of the 4^3, P = 3, Re 30 Taylor-Green state against
    the oracle evaluated in 80-bit extended precision (basis tables and
    constants too): within max(1e-12, 4 x the FP64 oracle's own distance from
    it) per variable."""
    import test_oracle_pins as pins
    dg, *_ = _oracle()
    say("residual C1 vs extended precision")
    prm = dg.Params(N=4, P=3, Re=30.0)
    q = dg.tgv_initial_condition(prm)
    floor, Rld = pins.roundoff_floor(q, prm)
    got, _ = _residual_case(B, 4, 3, 30.0, 0.0, True, dg.to_flat(q))
    ref = np.asarray(Rld, dtype=np.longdouble).reshape(5, -1)
    got = np.asarray(got, dtype=np.longdouble).reshape(5, -1)
    err = np.asarray(np.sqrt(np.sum((got - ref) ** 2, axis=1)) / np.sqrt(np.sum(ref ** 2, axis=1)), dtype=np.float64)
    print("device vs extended precision", err, "FP64 oracle floor", floor)
    assert np.all(err <= np.maximum(1e-12, 4.0 * floor)), (err, floor)


def test_stable_dt_viscous_branch(B):
    """Re = 1 on 4^3 elements: the viscous bound of Eq. (7) binds; the device
    value equals the oracle's (and its closed form)."""
    dg, *_ = _oracle()
    say("stable dt viscous")
    for N, P, Re in ((4, 3, 1.0), (4, 5, 0.5)):
        prm = dg.Params(N=N, P=P, Re=Re)
        q0 = dg.tgv_initial_condition(prm)
        ref = dg.stable_dt(q0, prm)
        closed = 0.4 * prm.h ** 2 / ((P + 1) ** 4 * prm.gamma * prm.mu / prm.Pr)
        assert abs(ref / closed - 1) < 1e-14
        m = B.Mesh(N, P, Re)
        q = _to_gpu(dg.to_flat(q0))
        dt = B.dg_stable_dt(m, q)
        assert abs(dt / ref - 1) < 1e-14, (N, P, Re, dt, ref)


def test_rk_steps_C1(B):
    """10 Runge-Kutta steps of the Re-30 TGV on 4^3 elements at P = 3, CFL 0.4."""
    dg, forcing, projection, rk = _oracle()
    say("rk C1")
    prm = dg.Params(N=4, P=3, Re=30.0)
    q0 = dg.tgv_initial_condition(prm)
    dt_ref = dg.stable_dt(q0, prm)
    m = B.Mesh(4, 3, 30.0)
    q = _to_gpu(dg.to_flat(q0))
    dt = B.dg_stable_dt(m, q)
    assert abs(dt / dt_ref - 1) < 1e-13
    k = m.field(0.0)
    B.dg_rk_step(m, q, k, dt, 10)
    torch.cuda.synchronize()
    ref = rk.integrate(q0, dt_ref, 10, lambda qq, t: dg.residual(qq, prm))
    l2, li = field_parity(q.cpu().numpy(), dg.to_flat(ref), 1e-12)
    assert np.all(l2 < 1e-12) and np.all(li < 1e-11), (l2, li)


@pytest.mark.parametrize("N,P,Cs", [(3, 4, 0.1), (2, 6, 0.0), (7, 8, 0.1)])
def test_rk_steps_random(B, N, P, Cs):
    dg, forcing, projection, rk = _oracle()
    say("rk random", N, P, Cs)
    prm = dg.Params(N=N, P=P, Re=100.0, Cs=Cs)
    q0 = dg.to_blocks(synthetic.random_state(N, P, seed=11, momentum=0.3), N, P)
    dt = 0.2 * dg.stable_dt(q0, prm)
    m = B.Mesh(N, P, 100.0, Cs=Cs)
    q = _to_gpu(dg.to_flat(q0))
    k = m.field(0.0)
    B.dg_rk_step(m, q, k, dt, 3)
    torch.cuda.synchronize()
    ref = rk.integrate(q0, dt, 3, lambda qq, t: dg.residual(qq, prm))
    l2, li = field_parity(q.cpu().numpy(), dg.to_flat(ref), 1e-12)
    assert np.all(l2 < 1e-12) and np.all(li < 1e-11), (l2, li)


def test_rk_full_size_conservation_and_determinism(B):
    """At 16^3, P = 6, Re 1600 with the closure: two steps conserve mass,
    momentum and energy to round-off, and a rerun is bitwise identical."""
    say("rk full size conservation")
    m = B.Mesh(16, 6, 1600.0, Cs=0.1)
    q = m.field()
    B.dg_init_tgv(m, q)
    q0 = q.clone()
    d0 = B.dg_diagnostics(m, q).cpu().numpy().copy()
    dt = B.dg_stable_dt(m, q)
    k = m.field(0.0)
    B.dg_rk_step(m, q, k, dt, 2)
    d1 = B.dg_diagnostics(m, q).cpu().numpy().copy()
    q2 = q0.clone()
    B.dg_rk_step(m, q2, k, dt, 2)
    torch.cuda.synchronize()
    assert torch.equal(q, q2)
    vol = (2 * np.pi) ** 3
    assert abs(d1[3] - d0[3]) < 1e-13 * vol
    assert np.max(np.abs(d1[4:7] - d0[4:7])) < 1e-13 * vol
    assert abs(d1[7] - d0[7]) < 1e-13 * abs(d0[7])
    assert d1[0] < d0[0]    # kinetic energy decays


@pytest.mark.parametrize("P", [3, 6, 8])
def test_profiled_steps_equal_plain_steps(B, P):
    """The measurement twin runs the same launches: the state after profiled
    steps is bitwise the state after plain steps, and every stage kernel
    reports a positive mean duration (the network's is 0 without a model)."""
    say("profiled steps", P)
    m = B.Mesh(8, P, 1600.0)
    q = m.field()
    B.dg_init_tgv(m, q)
    dt = B.dg_stable_dt(m, q)
    q2 = q.clone()
    k, k2 = m.field(0.0), m.field(0.0)
    B.dg_rk_step(m, q, k, dt, 3)
    prof = B.dg_profile_steps(m, q2, k2, dt, 3)
    torch.cuda.synchronize()
    assert torch.equal(q, q2) and torch.equal(k, k2)
    assert prof["traces"] > 0 and prof["grad"] > 0 and prof["resid"] > 0 and prof["net"] == 0


@pytest.mark.parametrize("N", [8, 16])
def test_profiled_corrected_steps_equal_plain_steps(B, N):
    """The same with the forcing network at every stage (P = 3); on 16^3
    elements the BR1 pass and the network run as one launch."""
    say("profiled corrected steps", N)
    dims = [320, 256, 256, 256, 320]
    norm = [1.0, 0.0, 0.0, 0.0, synthetic.TGV_ENERGY_LEVEL, 0.01, 1.0, 1.0, 1.0, 1.0,
            0.0, 0.0, 0.0, 0.0, 0.0, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3]
    model = B.Model(dims, B.pack_params(synthetic.mlp_init(dims, seed=0)), norm, train=False)
    m = B.Mesh(N, 3, 200.0)
    q = m.field()
    B.dg_init_tgv(m, q)
    dt = B.dg_stable_dt(m, q)
    q2 = q.clone()
    k, k2 = m.field(0.0), m.field(0.0)
    B.dg_rk_step(m, q, k, dt, 3, model=model)
    prof = B.dg_profile_steps(m, q2, k2, dt, 3, model=model)
    torch.cuda.synchronize()
    assert torch.equal(q, q2) and torch.equal(k, k2)
    assert prof["net"] > 0 and prof["resid"] > 0
    # the fused launch is timed as "net"
    assert (prof["grad"] == 0) if N == 16 else (prof["grad"] > 0)


def test_diagnostics_and_error_norm(B):
    dg, forcing, projection, rk = _oracle()
    say("diagnostics")
    N, P = 3, 4
    prm = dg.Params(N=N, P=P, Re=100.0)
    qb = dg.to_blocks(synthetic.random_state(N, P, seed=21), N, P)
    m = B.Mesh(N, P, 100.0)
    q = _to_gpu(dg.to_flat(qb))
    d = B.dg_diagnostics(m, q).cpu().numpy()
    assert abs(d[0] - dg.kinetic_energy(qb, prm)) < 1e-13 * abs(d[0])
    assert abs(d[1] - dg.max_wave_speed(qb, prm)) < 1e-14 * d[1]
    assert d[2] == np.min(qb[0])
    tot = dg.totals(qb, prm)
    assert np.max(np.abs(d[3:] - tot) / np.abs(tot)) < 1e-13
    qr = dg.to_blocks(synthetic.random_state(N, P, seed=22), N, P)
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    B.dg_error_inf(m, q, _to_gpu(dg.to_flat(qr)), out)
    assert np.array_equal(out.cpu().numpy(), dg.error_inf(qb, qr))


@pytest.mark.parametrize("Ps,Pd", [(8, 3), (6, 3), (8, 6), (4, 4)])
def test_filter(B, Ps, Pd):
    dg, forcing, projection, rk = _oracle()
    say("filter", Ps, Pd)
    N = 2
    src = np.random.default_rng(Ps * 10 + Pd).standard_normal((5, N ** 3, (Ps + 1) ** 3))
    ms, md = B.Mesh(N, Ps, 100.0), B.Mesh(N, Pd, 100.0)
    out = md.field(0.0)
    B.dg_project(ms, md, _to_gpu(src), out)
    ref = dg.to_flat(projection.project(dg.to_blocks(src, N, Ps), Ps, Pd))
    assert np.max(np.abs(out.cpu().numpy() - ref)) < 1e-13 * np.max(np.abs(ref))


def test_forcing_target(B):
    """Eq. (5) pairs from a P = 6 snapshot to P = 3, with the closure in the
    high-order operator (float32 rows)."""
    dg, forcing, projection, rk = _oracle()
    say("forcing target")
    N = 2
    prm_hi = dg.Params(N=N, P=6, Re=1600.0, Cs=0.1)
    prm_lo = dg.Params(N=N, P=3, Re=1600.0)
    qb = dg.tgv_initial_condition(prm_hi)
    qb = qb + 0.01 * np.random.default_rng(5).standard_normal(qb.shape) * np.array([0, 1, 1, 1, 0])[:, None, None, None, None, None, None]
    x_ref, y_ref = forcing.forcing_target(qb, prm_hi, prm_lo)
    hi, lo = B.Mesh(N, 6, 1600.0, Cs=0.1), B.Mesh(N, 3, 1600.0)
    x = torch.zeros((N ** 3, 320), dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    B.dg_forcing_target(hi, lo, _to_gpu(dg.to_flat(qb)), x, y)
    torch.cuda.synchronize()
    assert np.max(np.abs(x.cpu().numpy() - x_ref)) <= 1e-7 * np.max(np.abs(x_ref))
    assert rel_l2(y.cpu().numpy(), y_ref) < 1e-6
