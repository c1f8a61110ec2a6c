"""Learned corrective forcing on one GPU, end to end (Sec. 2.1 three steps,
Algorithm 1, Sec. 3.3 time frames, Sec. 3.4 effective acceleration / Table 2,
Sec. 3.5 transfer learning).

1. High-order evolution: P = 8 Taylor-Green run from t = 0; over the training
   window, at every snapshot interval dT the training pairs are appended to a
   device dataset, in one or both of two forms:
     "eq5":  the instantaneous target of Eq. (5), x = G q_8, y = G p_8(q_8) -
             p_LO(G q_8), at the end of the interval;
     "alg1": Algorithm 1's discrete increment over each low-order step dt,
             x = G q_8(t), y = (G q_8(t + dt) - q_LO(t + dt)) / dt, q_LO the
             uncorrected low-order step from G q_8(t).
   The filtered reference G q_8(t) is kept for the error of Eq. (9).
2. Training: the per-variable normalisation of the dataset, then epochs of
   shuffled minibatches of Adam on the MSE loss, on the GPU, for each network
   variant (target form, variables read and forced, activation), from a
   Gaussian initialisation or from another network's weights (retraining).
3. Low-order evolution from G q_8(t0): the low order without and with each
   network -- "stage" variants force every Runge-Kutta stage (Eq. (4)),
   "post" variants correct after each uncorrected step as Algorithm 1 does --
   and plain higher orders for the accuracy-time comparison.  All errors are
   measured on the low-order space: e_n = max |G_{P->LO} q_P - G_{8->LO} q_8|
   over the three momenta (Eq. (9)).

``run_study`` is one time frame; ``run_transfer`` trains on one frame (or
Reynolds number) and applies the network to another directly, after a short
retraining from its weights, and against a network trained there from
scratch.  Every step runs in libdgnn.so; this driver only sequences calls
and keeps time.  ``python -m paper_2207_11571_amd.study --help``.
"""
import argparse
import json
import math
import time

import numpy as np
import torch

from . import binding as B

HIDDEN = [256, 256, 256]
MOMENTUM = (1, 2, 3)
ALL = (0, 1, 2, 3, 4)
P_HO = 8


def _sync():
    torch.cuda.synchronize()


def variant(name, target="eq5", io="all", act="tanh", mode="stage", epochs=30, lr=1e-3, mask=(1, 1, 1, 1, 1),
            scaling="variable"):
    """One network to train and evaluate.  target: "eq5" or "alg1" pairs; io:
    "all" (reads and forces the five variables) or "momentum" (the paper's
    network, Sec. 2.2); mode: "stage" (forcing at every stage) or "post"
    (Algorithm 1's correction after each step); scaling: "variable" (one
    affine map per variable) or "node" (per node of the element, the paper's
    rescaling of the values at each node)."""
    return dict(name=name, target=target, io=io, act=act, mode=mode, epochs=epochs, lr=lr, mask=tuple(mask),
                scaling=scaling)


class Reference:
    """A P = 8 Taylor-Green run from t = 0 at one Reynolds number, advanced on
    demand with a fixed step (from the initial state: dT / n_hi).  cs_hi /
    cs_lo: Smagorinsky constants of the high-order scheme (and of the plain
    higher orders compared with it) and of the low-order scheme, 0 for none
    (Table 1 case 3: LES in the high order; 3b without, 3c with LES in the
    corrected low order)."""

    def __init__(self, N, Re, dT, P_lo, cfl=0.4, cs_hi=0.0, cs_lo=0.0):
        self.N, self.Re, self.dT, self.P_lo = N, Re, dT, P_lo
        self.cs_hi, self.cs_lo = cs_hi, cs_lo
        self.m_hi, self.m_lo = B.Mesh(N, P_HO, Re, Cs=cs_hi), B.Mesh(N, P_lo, Re, Cs=cs_lo)
        self.q = self.m_hi.field()
        B.dg_init_tgv(self.m_hi, self.q)
        q_lo = self.m_lo.field()
        B.dg_project(self.m_hi, self.m_lo, self.q, q_lo)
        # low-order steps per interval; high-order steps a multiple of them
        self.n_lo = math.ceil(dT / B.dg_stable_dt(self.m_lo, q_lo, cfl) - 1e-12)
        dt_hi = B.dg_stable_dt(self.m_hi, self.q, cfl)
        self.n_hi = self.n_lo * math.ceil(dT / self.n_lo / dt_hi - 1e-12)
        self.dt_hi = dT / self.n_hi
        self.k = self.m_hi.field(0.0)
        self.steps = 0          # intervals dT advanced
        self.seconds = 0.0

    @property
    def t(self):
        return self.steps * self.dT

    def advance_to(self, t_target):
        n = int(round(t_target / self.dT)) - self.steps
        if n < 0:
            raise ValueError("the reference cannot go back in time")
        _sync()
        ta = time.perf_counter()
        if n:
            B.dg_rk_step(self.m_hi, self.q, self.k, self.dt_hi, n * self.n_hi)
        _sync()
        self.seconds += time.perf_counter() - ta
        self.steps += n
        self.check()

    def check(self):
        d = B.dg_diagnostics(self.m_hi, self.q).cpu().numpy()
        if not np.all(np.isfinite(d)) or not d[2] > 0:
            raise FloatingPointError(f"P{P_HO} reference at Re={self.Re:g} is no longer finite at t={self.t:g}")

    def window(self, snapshots, n_eval, targets, orders=(), log=print):
        """From the current time: training pairs over the first `snapshots`
        intervals and the filtered reference over n_eval intervals."""
        m_hi, m_lo = self.m_hi, self.m_lo
        E, n_p = m_lo.E, m_lo.n_p
        t0 = self.t
        data = {}
        for tg in targets:
            rows = snapshots * E * (self.n_lo if tg == "alg1" else 1)
            data[tg] = (torch.empty((rows, 5 * n_p), dtype=torch.float32, device="cuda"),
                        torch.empty((rows, 5 * n_p), dtype=torch.float32, device="cuda"))
        ref = torch.empty((n_eval + 1, 5, E, n_p), dtype=torch.float64, device="cuda")
        init = {}
        for P in orders:
            m = B.Mesh(self.N, P, self.Re, Cs=self.cs_hi)
            f = m.field()
            B.dg_project(m_hi, m, self.q, f)
            init[P] = (m, f)
        B.dg_project(m_hi, m_lo, self.q, ref[0])
        ws_eq5 = ws_alg1 = None
        _sync()
        ta = time.perf_counter()
        for j in range(1, n_eval + 1):
            if j <= snapshots and "alg1" in data:
                X, Y = data["alg1"]
                for i in range(self.n_lo):
                    r0 = ((j - 1) * self.n_lo + i) * E
                    ws_alg1 = B.dg_increment_target(m_hi, m_lo, self.q, self.k, self.dT / self.n_lo,
                                                     self.n_hi // self.n_lo, X[r0:r0 + E], Y[r0:r0 + E], ws=ws_alg1)
            else:
                B.dg_rk_step(m_hi, self.q, self.k, self.dt_hi, self.n_hi)
            B.dg_project(m_hi, m_lo, self.q, ref[j])
            if j <= snapshots and "eq5" in data:
                X, Y = data["eq5"]
                ws_eq5 = B.dg_forcing_target(m_hi, m_lo, self.q, X[(j - 1) * E:j * E], Y[(j - 1) * E:j * E],
                                             ws=ws_eq5)
        _sync()
        t_gen = time.perf_counter() - ta
        self.seconds += t_gen
        self.steps += n_eval
        self.check()
        log(f"P{P_HO} Re={self.Re:g} window from t={t0:g}: {t_gen:.2f}s, datasets " +
            ", ".join(f"{k} {tuple(v[0].shape)}" for k, v in data.items()))
        return {"t0": t0, "data": data, "ref": ref, "init": init, "seconds": t_gen, "n_eval": n_eval,
                "snapshots": snapshots}


def train(X, Y, n_p, v, batch, seed=0, norm=None, init_params=None, log=print):
    """Trains one network variant on rows (X, Y); returns (model, norm,
    record).  norm: normalisation (default: the dataset's statistics);
    init_params: float32 device tensor of weights to start from (default:
    Gaussian)."""
    import synthetic
    rows = X.shape[0]
    nb = rows // batch
    io = MOMENTUM if v["io"] == "momentum" else ALL
    dims = [len(io) * n_p] + HIDDEN + [len(io) * n_p]
    flops = 3 * 2 * sum(a * b for a, b in zip(dims[:-1], dims[1:])) * batch
    if norm is None:
        norm = B.nn_data_stats(X, Y, n_p)
    params = init_params.clone() if init_params is not None else B.pack_params(synthetic.mlp_init(dims, seed=seed))
    model = B.Model(dims, params, norm, mask=v["mask"], activation=v["act"], in_vars=io, out_vars=io)
    if v.get("scaling", "variable") == "node":
        model.set_column_norm(B.nn_column_stats(X, Y, n_p), n_p)
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    _sync()
    ta = time.perf_counter()
    for ep in range(v["epochs"]):
        perm = torch.from_numpy(synthetic.epoch_permutation(rows, rng).astype(np.int32)).cuda()
        ep_loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        for b in range(nb):
            B.nn_train_step(model, X, Y, lr=v["lr"], loss=loss, idx=perm[b * batch:(b + 1) * batch])
            ep_loss += loss
        losses.append(float(ep_loss.item()) / nb)
    _sync()
    t_train = time.perf_counter() - ta
    rec = {**v, "pairs": rows, "batches_per_epoch": nb, "dims": dims, "seconds": t_train, "norm": list(norm),
           "steps_per_s": v["epochs"] * nb / t_train if t_train > 0 else None,
           "tflops": v["epochs"] * nb * flops / t_train / 1e12 if t_train > 0 else None,
           "loss_per_epoch": losses, "from_weights": init_params is not None}
    if losses:
        log(f"training {v['name']} ({v['target']} pairs, {v['io']}, {v['act']}, {v['mode']}"
            f"{', from given weights' if init_params is not None else ''}): {v['epochs']} epochs x {nb} batches "
            f"in {t_train:.2f}s, loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    return model, norm, rec


def evolve(ref, win, mesh, q0, window, model=None, mode="stage", cfl=0.4):
    """Low- or high-order run from q0 over the window's evaluation span; e_n
    against the filtered reference on the low-order space."""
    m_lo, dT, n_eval = ref.m_lo, ref.dT, win["n_eval"]
    q = q0.clone()
    k = mesh.field(0.0)
    n = ref.n_lo if mesh.P == ref.P_lo else math.ceil(dT / B.dg_stable_dt(mesh, q, cfl) - 1e-12)
    dt = dT / n
    step = B.dg_rk_step_post if mode == "post" else B.dg_rk_step
    tmp = m_lo.field()
    err = torch.empty(3, dtype=torch.float64, device="cuda")
    errs = []
    wall = 0.0
    for j in range(n_eval + 1):
        if j > 0:
            _sync()
            ta = time.perf_counter()
            step(mesh, q, k, dt, n, model=model)
            _sync()
            wall += time.perf_counter() - ta
        if mesh.P == ref.P_lo:
            B.dg_error_inf(mesh, q, win["ref"][j], err)
        else:
            B.dg_project(mesh, m_lo, q, tmp)
            B.dg_error_inf(m_lo, tmp, win["ref"][j], err)
        errs.append(err.cpu().numpy().tolist())
    e = np.array(errs)
    times = win["t0"] + dT * np.arange(n_eval + 1)
    inwin = (times > win["t0"]) & (times <= win["t0"] + window + 1e-9)
    beyond = times > win["t0"] + window + 1e-9
    span = dT * n_eval
    return {"P": mesh.P, "mode": mode if model is not None else None, "dt": dt, "steps": n * n_eval,
            "wall_s": wall, "wall_per_unit_time_s": wall / span,
            "dof_updates_per_s": mesh.E * mesh.n_p * 3 * n * n_eval / wall,
            "e_max_momentum": e.max(axis=1).tolist(), "times": times.tolist(),
            "mean_e_window": float(e[inwin].max(axis=1).mean()),
            "mean_e_beyond": float(e[beyond].max(axis=1).mean()) if beyond.any() else None,
            "final_e": float(e[-1].max())}


def _gain(base, run):
    e0, e1 = np.array(base["e_max_momentum"]), np.array(run["e_max_momentum"])
    worse = np.nonzero(e1[1:] > e0[1:])[0]
    return {"window_ratio": run["mean_e_window"] / base["mean_e_window"],
            "beyond_ratio": (run["mean_e_beyond"] / base["mean_e_beyond"]) if base["mean_e_beyond"] else None,
            "better_than_uncorrected_until": base["times"][1 + worse[0]] if len(worse) else base["times"][-1]}


def run_study(N=16, Re=1600.0, t0=4.0, window=1.0, snapshots=50, eval_end=5.5, epochs=30, batch=4096,
              lr=1e-3, seed=0, orders=(4, 5, 6), cfl=0.4, log=print, variants=None, P_lo=3, cs_hi=0.0, cs_lo=0.0):
    """One time frame.  variants: list of ``variant(...)`` dicts (or (name,
    mask, epochs, lr) tuples: Eq. (5) pairs, all variables, tanh, every
    stage); default one such variant from the arguments.  cs_hi, cs_lo: the
    Smagorinsky constants of the high- and low-order schemes (0: none)."""
    if variants is None:
        variants = [variant("nn", epochs=epochs, lr=lr)]
    variants = [v if isinstance(v, dict) else variant(v[0], mask=v[1], epochs=v[2], lr=v[3]) for v in variants]
    targets = sorted({v["target"] for v in variants})
    out = {"config": dict(N=N, Re=Re, t0=t0, window=window, snapshots=snapshots, eval_end=eval_end, P_lo=P_lo,
                          batch=batch, seed=seed, orders=list(orders), variants=variants, cs_hi=cs_hi,
                          cs_lo=cs_lo)}
    dT = window / snapshots
    n_eval = int(round((eval_end - t0) / dT))
    lo = f"P{P_lo}"

    ref = Reference(N, Re, dT, P_lo, cfl, cs_hi, cs_lo)
    ref.advance_to(t0)
    t_ref = ref.seconds
    log(f"P{P_HO} reached t0={t0} in {t_ref:.2f}s (dt={ref.dt_hi:.4e})")
    win = ref.window(snapshots, n_eval, targets, orders, log)
    out["reference"] = {"P": P_HO, "dt": ref.dt_hi, "seconds_to_t0": t_ref, "seconds_window_and_eval": win["seconds"],
                        "wall_per_unit_time_s": win["seconds"] / (eval_end - t0),
                        "low_order_steps_per_snapshot": ref.n_lo}

    n_p = ref.m_lo.n_p
    norms = {tg: B.nn_data_stats(X, Y, n_p) for tg, (X, Y) in win["data"].items()}
    models = {}
    out["training"] = {"norm": norms, "variants": {}}
    for v in variants:
        X, Y = win["data"][v["target"]]
        model, _, rec = train(X, Y, n_p, v, batch, seed, norm=norms[v["target"]], log=log)
        models[v["name"]] = (model, v["mode"])
        out["training"]["variants"][v["name"]] = rec

    runs = {lo: evolve(ref, win, ref.m_lo, win["ref"][0], window, cfl=cfl)}
    for name, (model, mode) in models.items():
        runs[f"{lo}+{name}"] = evolve(ref, win, ref.m_lo, win["ref"][0], window, model, mode, cfl)
    for P, (m, f) in win["init"].items():
        runs[f"P{P}"] = evolve(ref, win, m, f, window, cfl=cfl)
    out["runs"] = runs
    for name, r in runs.items():
        log(f"{name:8s} dt={r['dt']:.3e} wall/unit time={r['wall_per_unit_time_s']:.3f}s "
            f"mean e window={r['mean_e_window']:.3e} beyond={r['mean_e_beyond']} final={r['final_e']:.3e}")
    out["gain"], out["comparison"] = {}, {}
    for name in models:
        r = runs[f"{lo}+{name}"]
        out["gain"][name] = _gain(runs[lo], r)
        out["comparison"][name] = {
            f"P{P}": {"wall_ratio_vs_corrected": runs[f"P{P}"]["wall_s"] / r["wall_s"],
                      "error_ratio_corrected_vs_window": r["mean_e_window"] / runs[f"P{P}"]["mean_e_window"],
                      "error_ratio_corrected_vs_beyond": (r["mean_e_beyond"] / runs[f"P{P}"]["mean_e_beyond"])
                      if runs[f"P{P}"]["mean_e_beyond"] else None}
            for P in win["init"]}
    return out


def run_transfer(N=8, P_lo=3, source=(1600.0, 4.0), target=(1600.0, 7.0), window=0.15, snapshots=100,
                 eval_span=0.3, net=None, retrain_epochs=50, batch=512, seed=0, cfl=0.4, log=print):
    """Transfer learning (Sec. 3.5): a network trained on the source frame
    (Re, t0) is applied to the target frame (Re, t0) as it is ("source"),
    after `retrain_epochs` epochs of retraining on the target pairs starting
    from its weights and keeping its normalisation ("retrained"), and
    compared with a network trained on the target pairs from a Gaussian
    initialisation for the full epoch count ("scratch") and with the
    uncorrected low order."""
    net = net or variant("alg1a", "alg1", "all", "tanh", "post", epochs=200)
    dT = window / snapshots
    n_eval = int(round(eval_span / dT))
    lo = f"P{P_lo}"
    out = {"config": dict(N=N, P_lo=P_lo, source=list(source), target=list(target), window=window,
                          snapshots=snapshots, eval_span=eval_span, net=net, retrain_epochs=retrain_epochs,
                          batch=batch, seed=seed)}
    refs = {}

    def frame(Re, t0):
        if Re not in refs:
            refs[Re] = Reference(N, Re, dT, P_lo, cfl)
        ref = refs[Re]
        ref.advance_to(t0)
        return ref, ref.window(snapshots, n_eval, [net["target"]], (), log)

    ref_s, win_s = frame(*source)
    n_p = ref_s.m_lo.n_p
    X, Y = win_s["data"][net["target"]]
    src_model, src_norm, src_rec = train(X, Y, n_p, net, batch, seed, log=log)
    del win_s
    ref_t, win_t = frame(*target)
    X, Y = win_t["data"][net["target"]]
    scratch, _, scr_rec = train(X, Y, n_p, {**net, "name": "scratch"}, batch, seed, log=log)
    retrained, _, ret_rec = train(X, Y, n_p, {**net, "name": "retrained", "epochs": retrain_epochs}, batch, seed,
                                  norm=src_norm, init_params=src_model.params, log=log)
    out["training"] = {"source": src_rec, "scratch": scr_rec, "retrained": ret_rec}
    runs = {lo: evolve(ref_t, win_t, ref_t.m_lo, win_t["ref"][0], window, cfl=cfl)}
    for name, model in (("source", src_model), ("retrained", retrained), ("scratch", scratch)):
        runs[f"{lo}+{name}"] = evolve(ref_t, win_t, ref_t.m_lo, win_t["ref"][0], window, model, net["mode"], cfl)
    out["runs"] = runs
    for name, r in runs.items():
        log(f"{name:14s} mean e window={r['mean_e_window']:.3e} beyond={r['mean_e_beyond']} final={r['final_e']:.3e}")
    out["gain"] = {name: _gain(runs[lo], runs[f"{lo}+{name}"]) for name in ("source", "retrained", "scratch")}
    out["training_seconds"] = {"scratch": scr_rec["seconds"], "retrained": ret_rec["seconds"]}
    return out


def run_online(N=8, Re=200.0, P_lo=3, t0=4.0, t_end=7.0, window=0.15, snapshots=100, retrain_window=0.075,
               retrain_snapshots=50, tol=1e-2, max_retrains=50, net=None, retrain_epochs=50, batch=512, seed=0,
               cfl=0.4, log=print):
    """The online retraining loop the paper proposes as future work (Sec. 4):
    a P = 8 shadow run supplies the reference for the error; the corrected low-order run
    starts from the filtered P = 8 state at the end of the first training
    window, and whenever its error e_n exceeds `tol`, the shadow's next
    `retrain_window` produces fresh pairs, the network is retrained from its
    current weights for `retrain_epochs` epochs, and the low-order state is
    set to the filtered P = 8 state again (Algorithm 1's matching step).
    Compared, from the same start, with: the first network never retrained
    but re-matched at the same times ("rematched"), the first network alone
    ("fixed"), and the uncorrected low order."""
    net = net or variant("alg1a", "alg1", "all", "tanh", "post", epochs=200)
    dT = window / snapshots
    ref = Reference(N, Re, dT, P_lo, cfl)
    ref.advance_to(t0)
    win = ref.window(snapshots, snapshots, [net["target"]], (), log)
    n_p = ref.m_lo.n_p
    X, Y = win["data"][net["target"]]
    model, norm, rec0 = train(X, Y, n_p, net, batch, seed, log=log)
    fixed = model          # retraining builds new models from copies of the weights
    del win
    m_lo = ref.m_lo
    step = B.dg_rk_step_post if net["mode"] == "post" else B.dg_rk_step
    dt = dT / ref.n_lo
    names = ("online", "rematched", "fixed", "uncorrected")
    q = {nm: m_lo.field() for nm in names}
    B.dg_project(ref.m_hi, m_lo, ref.q, q["online"])
    for nm in names[1:]:
        q[nm].copy_(q["online"])
    k = m_lo.field(0.0)
    g = m_lo.field()
    err = torch.empty(3, dtype=torch.float64, device="cuda")

    def advance(nm, n):
        mdl = {"online": model, "rematched": fixed, "fixed": fixed, "uncorrected": None}[nm]
        if mdl is None:
            B.dg_rk_step(m_lo, q[nm], k, dt, n)
        else:
            step(m_lo, q[nm], k, dt, n, model=mdl)

    hist = {"t": [], **{nm: [] for nm in names}}
    events = []
    seconds = {"low_order": 0.0, "reference": 0.0, "retraining": 0.0}
    t_ho = 0.0
    while ref.t < t_end - 1e-9:
        _sync()
        ta = time.perf_counter()
        advance("online", ref.n_lo)
        _sync()
        seconds["low_order"] += time.perf_counter() - ta
        for nm in names[1:]:
            advance(nm, ref.n_lo)
        s0 = ref.seconds
        ref.advance_to(ref.t + dT)
        seconds["reference"] += ref.seconds - s0
        B.dg_project(ref.m_hi, m_lo, ref.q, g)
        hist["t"].append(ref.t)
        for nm in names:
            B.dg_error_inf(m_lo, q[nm], g, err)
            hist[nm].append(float(err.max().item()))
        e_on = hist["online"][-1]
        if e_on > tol and len(events) < max_retrains and ref.t + retrain_window < t_end:
            s0 = ref.seconds
            w = ref.window(retrain_snapshots, retrain_snapshots, [net["target"]], (), log)
            seconds["reference"] += ref.seconds - s0
            t_ho += retrain_window
            X, Y = w["data"][net["target"]]
            model, _, rec = train(X, Y, n_p, {**net, "name": "online", "epochs": retrain_epochs}, batch, seed,
                                  norm=norm, init_params=model.params, log=log)
            seconds["retraining"] += rec["seconds"]
            del w
            B.dg_project(ref.m_hi, m_lo, ref.q, q["online"])
            q["rematched"].copy_(q["online"])
            for nm in ("fixed", "uncorrected"):     # they cross the high-order window unchanged in kind
                advance(nm, ref.n_lo * retrain_snapshots)
            events.append({"t": ref.t, "e_before": e_on, "train_s": rec["seconds"]})
            log(f"retrained at t={ref.t:.4f} (e_n {e_on:.3e} > {tol:g})")
    arr = {nm: np.array(hist[nm]) for nm in names}
    out = {"config": dict(N=N, Re=Re, P_lo=P_lo, t0=t0, t_end=t_end, window=window, snapshots=snapshots,
                          retrain_window=retrain_window, tol=tol, retrain_epochs=retrain_epochs, net=net),
           "history": hist, "retrains": events, "seconds": seconds, "initial_training_s": rec0["seconds"],
           "high_order_fraction_of_span": t_ho / (t_end - t0 - window),
           "mean_e": {nm: float(arr[nm].mean()) for nm in names},
           "max_e": {nm: float(arr[nm].max()) for nm in names},
           "final_e": {nm: float(arr[nm][-1]) for nm in names}}
    log(f"online loop to t={ref.t:.3f}: {len(events)} retrains; mean e_n " +
        ", ".join(f"{nm} {out['mean_e'][nm]:.3e}" for nm in names))
    return out


def _variants(spec):
    out = []
    for item in spec.split(";"):
        f = item.split(":")
        name, target, io, act, mode, ep, lr = f[:7]
        out.append(variant(name, target, io, act, mode, int(ep), float(lr),
                           scaling=f[7] if len(f) > 7 else "variable"))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=16)
    ap.add_argument("--Re", type=float, default=1600.0)
    ap.add_argument("--P-lo", type=int, default=3)
    ap.add_argument("--t0", type=float, default=4.0)
    ap.add_argument("--window", type=float, default=1.0)
    ap.add_argument("--snapshots", type=int, default=50)
    ap.add_argument("--eval-end", type=float, default=5.5)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--orders", default="4,5,6")
    ap.add_argument("--out", default=None)
    ap.add_argument("--variants", default=None,
                    help="semicolon list name:target:io:act:mode:epochs:lr, e.g. "
                         "nn:eq5:all:tanh:stage:30:1e-3;alg1:alg1:momentum:relu:post:30:1e-3")
    ap.add_argument("--transfer", default=None,
                    help="Re_source,t0_source,Re_target,t0_target: transfer-learning run instead of one frame")
    ap.add_argument("--retrain-epochs", type=int, default=50)
    ap.add_argument("--online", default=None, help="t0,t_end: online retraining loop instead of one frame")
    ap.add_argument("--tol", type=float, default=1e-2)
    ap.add_argument("--eval-span", type=float, default=0.3)
    ap.add_argument("--cs-hi", type=float, default=0.0, help="Smagorinsky constant of the high order (0: none)")
    ap.add_argument("--cs-lo", type=float, default=0.0, help="Smagorinsky constant of the low order (0: none)")
    a = ap.parse_args()
    torch.cuda.set_device(0)
    log = lambda *x: print("[study]", *x, flush=True)
    if a.online:
        t0, t_end = (float(x) for x in a.online.split(","))
        net = _variants(a.variants)[0] if a.variants else None
        res = run_online(N=a.N, Re=a.Re, P_lo=a.P_lo, t0=t0, t_end=t_end, window=a.window, snapshots=a.snapshots,
                         tol=a.tol, net=net, retrain_epochs=a.retrain_epochs, batch=a.batch, log=log)
        summary = {k: res[k] for k in ("mean_e", "max_e", "final_e", "retrains", "seconds",
                                       "high_order_fraction_of_span")}
    elif a.transfer:
        rs, ts, rt, tt = (float(x) for x in a.transfer.split(","))
        net = _variants(a.variants)[0] if a.variants else None
        res = run_transfer(N=a.N, P_lo=a.P_lo, source=(rs, ts), target=(rt, tt), window=a.window,
                           snapshots=a.snapshots, eval_span=a.eval_span, net=net, retrain_epochs=a.retrain_epochs,
                           batch=a.batch, log=log)
        summary = {"gain": res["gain"], "training_seconds": res["training_seconds"]}
    else:
        res = run_study(N=a.N, Re=a.Re, t0=a.t0, window=a.window, snapshots=a.snapshots, eval_end=a.eval_end,
                        epochs=a.epochs, batch=a.batch, lr=a.lr, orders=tuple(int(x) for x in a.orders.split(",")),
                        log=log, variants=_variants(a.variants) if a.variants else None, P_lo=a.P_lo,
                        cs_hi=a.cs_hi, cs_lo=a.cs_lo)
        summary = {"gain": res["gain"], "comparison": res["comparison"]}
    if a.out:
        open(a.out, "w").write(json.dumps(res))
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
