"""GPU tests of the continuous-batching solve server (solve_submit /
solve_poll through the C ABI): each solve computes the same result alone and
in a mix, admission respects the arena, impossible requests fail at once,
a non-finite solve fails alone."""
import time

import numpy as np
import pytest

import synthetic
from helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DIMS = [320, 256, 256, 256, 320]
NORM = [1.0, 0.0, 0.0, 0.0, synthetic.TGV_ENERGY_LEVEL, 0.01, 1, 1, 1, 1, 0, 0, 0, 0, 0, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3]


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_11571_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def model(B):
    return B.Model(DIMS, B.pack_params(synthetic.mlp_init(DIMS, seed=0)), NORM, train=False)


def _wait(srv, ids, timeout=120.0):
    t0 = time.time()
    out = {}
    while len(out) < len(ids):
        for i in ids:
            if i in out:
                continue
            rc, st = srv.poll(i)
            if rc == 0:
                out[i] = st
        if time.time() - t0 > timeout:
            raise TimeoutError(f"solves not finished: {set(ids) - set(out)}")
        time.sleep(0.01)
    return out


MIX = [
    dict(Re=200.0, P=3, N=4, use_nn=True),
    dict(Re=1600.0, P=6, N=4),
    dict(Re=30.0, P=3, N=8),
    dict(Re=1600.0, P=8, N=4, Cs=0.1),
    dict(Re=200.0, P=3, N=8, use_nn=True),
    dict(Re=30.0, P=6, N=2),
    dict(Re=200.0, P=3, N=4, use_nn=True, after_step=True),
    # with the P = 8 solve above, 407 elements of two solves in one P = 8
    # launch
    dict(Re=1600.0, P=8, N=7),
]


def test_alone_equals_mix(B, model):
    say("serving alone vs mix")
    t_end = 0.02
    alone = []
    for r in MIX:
        srv = B.Server(256 << 20, max_slots=8)
        rid = srv.submit(t_end=t_end, model=model if r.get("use_nn") else None, ke_every=1, ke_capacity=4096,
                         want_state=True, **r)
        st = _wait(srv, [rid])[rid]
        assert st.state == B.SOLVE_DONE, st.error
        ke, q = srv.results(rid)
        alone.append((q.copy(), ke[:2 * st.ke_count].copy()))
        srv.close()
    srv = B.Server(1 << 30, max_slots=16)
    ids = []
    for j, r in enumerate(MIX):
        ids.append(srv.submit(t_end=t_end, model=model if r.get("use_nn") else None, ke_every=1, ke_capacity=4096,
                              want_state=True, **r))
        if j == 2:
            time.sleep(0.05)     # later requests arrive while the first ones run
    sts = _wait(srv, ids)
    for rid, (q_alone, ke_alone) in zip(ids, alone):
        assert sts[rid].state == B.SOLVE_DONE
        ke, q = srv.results(rid)
        assert np.array_equal(q, q_alone)
        assert np.array_equal(ke[:2 * sts[rid].ke_count], ke_alone)
        assert sts[rid].latency_s > 0
    busy, batches = srv.stats()
    assert batches > 0 and busy > 0
    srv.close()


def test_admission_under_small_arena(B):
    say("serving admission")
    foot = B.solve_footprint(6, 4)
    srv = B.Server(foot + (foot // 2), max_slots=8)     # room for one solve at a time
    ids = [srv.submit(Re=1600.0, P=6, N=4, t_end=0.01) for _ in range(3)]
    sts = _wait(srv, ids)
    assert all(s.state == B.SOLVE_DONE for s in sts.values())
    queued = sorted(s.queue_s for s in sts.values())
    assert queued[-1] > queued[0]          # later ones waited for a slot
    with pytest.raises(B.DGError) as ei:
        srv.submit(Re=1600.0, P=8, N=16, t_end=0.01)     # can never fit
    assert ei.value.code == B.DG_ENOSPC
    srv.close()


def test_nonfinite_solve_fails_alone(B):
    say("serving nan injection")
    srv = B.Server(256 << 20, max_slots=8)
    bad = srv.submit(Re=200.0, P=3, N=4, t_end=0.5, ke_every=1)
    good = srv.submit(Re=200.0, P=3, N=4, t_end=0.05, ke_every=1)
    srv.inject_nan(bad)
    sts = _wait(srv, [bad, good])
    assert sts[bad].state == B.SOLVE_FAILED and sts[bad].error == B.DG_ENONFINITE
    assert sts[good].state == B.SOLVE_DONE
    srv.close()


def test_invalid_requests(B):
    srv = B.Server(64 << 20, max_slots=2)
    with pytest.raises(B.DGError):
        srv.submit(Re=200.0, P=9, N=4, t_end=0.1)
    with pytest.raises(B.DGError):
        srv.submit(Re=200.0, P=3, N=4, t_end=0.1, use_nn=True, model=None)
    with pytest.raises(B.DGError):
        srv.submit(Re=-1.0, P=3, N=4, t_end=0.1)
    srv.close()


SERVED = {"P3 forcing every stage": dict(Re=200.0, P=3, N=4, Cs=0.0, use_nn=True, after_step=False, t_end=0.03),
          # 16^3: the library fuses the BR1 pass and the network, the server does not
          "P3 forcing every stage, 16^3": dict(Re=200.0, P=3, N=16, Cs=0.0, use_nn=True, after_step=False,
                                               t_end=0.004),
          "P3 correction after each step": dict(Re=200.0, P=3, N=4, Cs=0.0, use_nn=True, after_step=True,
                                                t_end=0.03),
          "P6 plain": dict(Re=1600.0, P=6, N=3, Cs=0.0, use_nn=False, after_step=False, t_end=0.005),
          "P8 plain with the closure": dict(Re=1600.0, P=8, N=2, Cs=0.1, use_nn=False, after_step=False,
                                            t_end=0.003)}


@pytest.mark.parametrize("case", list(SERVED))
def test_server_solve_equals_library_stepping(B, model, case):
    """A solve run by the server (plain, forcing at every stage, or Algorithm
    1's correction after each step) ends in the same state as the library's
    own stepper with the same time step, bitwise."""
    c = SERVED[case]
    say("serving vs library stepping", case)
    srv = B.Server(256 << 20, max_slots=4)
    kw = dict(use_nn=True, model=model, after_step=c["after_step"]) if c["use_nn"] else {}
    if c["Cs"]:
        kw["Cs"] = c["Cs"]
    rid = srv.submit(Re=c["Re"], P=c["P"], N=c["N"], t_end=c["t_end"], want_state=True, **kw)
    st = _wait(srv, [rid])[rid]
    assert st.state == B.SOLVE_DONE, st.error
    _, q_srv = srv.results(rid)
    srv.close()
    m = B.Mesh(c["N"], c["P"], c["Re"], Cs=c["Cs"])
    q = m.field()
    B.dg_init_tgv(m, q)
    k = m.field(0.0)
    assert st.n_steps >= 1 and abs(st.dt * st.n_steps - c["t_end"]) < 1e-12
    step = B.dg_rk_step_post if c["after_step"] else B.dg_rk_step
    step(m, q, k, st.dt, st.n_steps, model=model if c["use_nn"] else None)
    torch.cuda.synchronize()
    assert np.array_equal(q.cpu().numpy().ravel(), q_srv)


ORACLE_SERVED = {"P3 with the network at every stage": dict(Re=200.0, P=3, N=4, use_nn=True, t_end=0.03),
                 "P6 plain": dict(Re=1600.0, P=6, N=4, use_nn=False, t_end=0.006)}


@pytest.mark.parametrize("case", list(ORACLE_SERVED))
def test_served_solve_matches_oracle(B, model, case):
    """A solve run through solve_submit / solve_poll against the CPU oracle's
    own integration of the same problem (Taylor-Green state, Eq. (7) step
    from the initial state, RK3 of Eq. (3) or, with the network, Eq. (4)):
    final state per variable to 1e-12 relative for the plain solve and 1e-5
    for the corrected one (its bf16 forcing is ~1e-3 of the residual and
    agrees to 1e-2), the momenta measured against the momentum vector's norm;
    kinetic-energy record to 1e-3 (corrected) and 1e-12."""
    from oracle import dg, forcing, mlp, rk
    from helpers import state_parity
    c = ORACLE_SERVED[case]
    say("served solve vs oracle", case)
    srv = B.Server(256 << 20, max_slots=4)
    kw = dict(use_nn=True, model=model) if c["use_nn"] else {}
    rid = srv.submit(Re=c["Re"], P=c["P"], N=c["N"], t_end=c["t_end"], ke_every=1, ke_capacity=4096,
                     want_state=True, **kw)
    st = _wait(srv, [rid])[rid]
    assert st.state == B.SOLVE_DONE, st.error
    ke, q_srv = srv.results(rid)
    ke = ke[:2 * st.ke_count].reshape(-1, 2)
    srv.close()
    prm = dg.Params(N=c["N"], P=c["P"], Re=c["Re"])
    q0 = dg.tgv_initial_condition(prm)
    n_ref, dt_ref = dg.steps_for(c["t_end"], dg.stable_dt(q0, prm))
    assert st.n_steps == n_ref and abs(st.dt / dt_ref - 1) < 1e-13
    if c["use_nn"]:
        params = [(mlp.bf16_round(W), b.astype(np.float64)) for W, b in synthetic.mlp_init(DIMS, seed=0)]
        norm = forcing.Normalisation(NORM[0:5], NORM[5:10], NORM[10:15], NORM[15:20])
        rhs = lambda qq, t: forcing.corrected_rhs(qq, prm, params, norm)
    else:
        rhs = lambda qq, t: dg.residual(qq, prm)
    ke_ref = {0: dg.kinetic_energy(q0, prm)}
    q_ref = rk.integrate(q0, dt_ref, n_ref, rhs,
                         callback=lambda n, qq: ke_ref.__setitem__(n, dg.kinetic_energy(qq, prm)))
    l2, li = state_parity(q_srv, dg.to_flat(q_ref))
    tol = 1e-5 if c["use_nn"] else 1e-12
    print(case, "state rel L2", l2, "rel inf", li)
    assert np.all(l2 < tol) and np.all(li < 10 * tol), (l2, li)
    assert len(ke) >= n_ref
    errs = []
    for t, e in ke:
        n = int(round(t / dt_ref))
        assert abs(n * dt_ref - t) < 1e-9 and n in ke_ref
        errs.append(abs(e - ke_ref[n]) / ke_ref[n])
    print(case, "KE record max rel", max(errs))
    assert max(errs) < (1e-3 if c["use_nn"] else 1e-12)


def _served(B, srv, **kw):
    rid = srv.submit(ke_every=1, ke_capacity=4096, want_state=True, **kw)
    st = _wait(srv, [rid])[rid]
    ke, q = srv.results(rid)
    return st, ke[:2 * st.ke_count].reshape(-1, 2), q


def test_fallback_after_blow_up(B):
    """A network with absurd weights (x20, output scale 10) drives the
    corrected solve to blow up within its first round of steps: the server
    returns it to the initial state and finishes it uncorrected, so its
    final state equals the plain low-order stepping from the Taylor-Green
    state, bitwise, and its status says so."""
    say("serving fallback after blow-up")
    layers = [(20.0 * W, b + 0.5) for W, b in synthetic.mlp_init(DIMS, seed=0)]
    norm = list(NORM[:15]) + [10.0] * 5
    bad = B.Model(DIMS, B.pack_params(layers), norm, train=False)
    srv = B.Server(256 << 20, max_slots=4)
    st, ke, q_srv = _served(B, srv, Re=200.0, P=3, N=4, t_end=0.05, use_nn=True, model=bad)
    srv.close()
    assert st.state == B.SOLVE_DONE, st.error
    assert st.fallback == 1 and st.fallback_step == 0
    assert np.all(np.isfinite(q_srv)) and np.all(np.isfinite(ke))
    m = B.Mesh(4, 3, 200.0)
    q = m.field()
    B.dg_init_tgv(m, q)
    k = m.field(0.0)
    B.dg_rk_step(m, q, k, st.dt, st.n_steps)
    torch.cuda.synchronize()
    assert np.array_equal(q.cpu().numpy().ravel(), q_srv)
    # the record continues from the initial state with the uncorrected run
    assert len(ke) == st.n_steps + 1 and np.all(np.diff(ke[:, 0]) > 0)


def test_fallback_continues_from_the_last_checked_state(B):
    """A constant forcing of the x-momentum (0.2 per unit time, from a
    network whose only non-zero parameters are output biases) adds kinetic
    energy faster than the Re-200 flow dissipates it: the oracle puts the
    rise past 1e-3 of the initial value at step 61 on 4^3 elements, P = 3.
    The server falls back to the copy taken at the start of the round that
    crossed, and the final state equals the library's corrected stepping up
    to that step followed by uncorrected stepping to the end, bitwise."""
    say("serving fallback from a later round")
    layers = [(0.0 * W, 0.0 * b) for W, b in synthetic.mlp_init(DIMS, seed=0)]
    layers[-1][1][64:128] = 1.0
    norm = list(NORM[:15]) + [1e-3, 0.2, 1e-3, 1e-3, 1e-3]
    drift = B.Model(DIMS, B.pack_params(layers), norm, train=False)
    srv = B.Server(256 << 20, max_slots=4)
    st, ke, q_srv = _served(B, srv, Re=200.0, P=3, N=4, t_end=0.4, use_nn=True, model=drift)
    srv.close()
    assert st.state == B.SOLVE_DONE, st.error
    print("fallback from step", st.fallback_step, "of", st.n_steps)
    assert st.fallback == 1 and 0 < st.fallback_step <= 61
    m = B.Mesh(4, 3, 200.0)
    q = m.field()
    B.dg_init_tgv(m, q)
    k = m.field(0.0)
    B.dg_rk_step(m, q, k, st.dt, st.fallback_step, model=drift)
    B.dg_rk_step(m, q, k, st.dt, st.n_steps - st.fallback_step)
    torch.cuda.synchronize()
    assert np.array_equal(q.cpu().numpy().ravel(), q_srv)
    ke0 = ke[0, 1]
    assert np.all(ke[:, 1] <= ke0 * (1 + 1e-3))
    assert len(ke) == st.n_steps + 1


def test_healthy_corrected_solve_does_not_fall_back(B, model):
    say("serving no fallback for a healthy corrected solve")
    srv = B.Server(256 << 20, max_slots=4)
    st, ke, _ = _served(B, srv, Re=200.0, P=3, N=4, t_end=0.1, use_nn=True, model=model)
    srv.close()
    assert st.state == B.SOLVE_DONE and st.fallback == 0 and st.fallback_step == -1
