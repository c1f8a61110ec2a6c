"""Learned corrective forcing on one GPU, end to end (Sec. 2.1 three steps,
Algorithm 1, Sec. 3.3 time frames, Sec. 3.4 effective acceleration / Table 2).

1. High-order evolution: P = 8 Taylor-Green run from t = 0; over the training
   window, at every snapshot interval dT the training pairs are appended to a
   device dataset, in one or both of two forms:
     "eq5":  the instantaneous target of Eq. (5), x = G q_8, y = G p_8(q_8) -
             p_3(G q_8), at the end of the interval;
     "alg1": Algorithm 1's discrete increment over one low-order step dT,
             x = G q_8(t), y = (G q_8(t + dT) - q_3(t + dT)) / dT, q_3 the
             uncorrected low-order step from G q_8(t).
   The filtered reference G q_8(t) is kept for the error of Eq. (9).
2. Training: the per-variable normalisation of the dataset, then epochs of
   shuffled minibatches of Adam on the MSE loss, on the GPU, for each network
   variant (target form, variables read and forced, activation).
3. Low-order evolution from G q_8(t0): P = 3 without and with each network --
   "stage" variants force every Runge-Kutta stage (Eq. (4)), "post" variants
   correct after each uncorrected step as Algorithm 1 does -- and plain
   P = 4, 5, 6 for the accuracy-time comparison.  All errors are measured on
   the P = 3 space: e_n = max |G_{P->3} q_P - G_{8->3} q_8| over the three
   momenta (Eq. (9)).

Every step runs in libdgnn.so; this driver only sequences calls and keeps
time.  ``python -m paper_2207_11571_amd.study --help``.
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


def _sync():
    torch.cuda.synchronize()


def variant(name, target="eq5", io="all", act="tanh", mode="stage", epochs=30, lr=1e-3, mask=(1, 1, 1, 1, 1)):
    """One network to train and evaluate.  target: "eq5" or "alg1" pairs; io:
    "all" (reads and forces the five variables) or "momentum" (the paper's
    network, Sec. 2.2); mode: "stage" (forcing at every stage) or "post"
    (Algorithm 1's correction after each step)."""
    return dict(name=name, target=target, io=io, act=act, mode=mode, epochs=epochs, lr=lr, mask=tuple(mask))


def run_study(N=16, Re=1600.0, t0=4.0, window=1.0, snapshots=50, eval_end=5.5, epochs=30, batch=4096,
              lr=1e-3, seed=0, orders=(4, 5, 6), cfl=0.4, log=print, variants=None):
    """variants: list of ``variant(...)`` dicts (or (name, mask, epochs, lr)
    tuples: Eq. (5) pairs, all variables, tanh, every stage); default one
    such variant from the arguments."""
    if variants is None:
        variants = [variant("nn", epochs=epochs, lr=lr)]
    variants = [v if isinstance(v, dict) else variant(v[0], mask=v[1], epochs=v[2], lr=v[3]) for v in variants]
    targets = sorted({v["target"] for v in variants})
    import synthetic
    out = {"config": dict(N=N, Re=Re, t0=t0, window=window, snapshots=snapshots, eval_end=eval_end,
                          batch=batch, seed=seed, orders=list(orders), variants=variants)}
    dT = window / snapshots
    n_eval = int(round((eval_end - t0) / dT))

    # ---------------------------------------------------------------- step 1
    m8, m3 = B.Mesh(N, 8, Re), B.Mesh(N, 3, Re)
    q8 = m8.field()
    B.dg_init_tgv(m8, q8)
    # the low-order step inside an interval (Algorithm 1's pairs are per low-order step)
    q3 = m3.field()
    B.dg_project(m8, m3, q8, q3)
    n3 = math.ceil(dT / B.dg_stable_dt(m3, q3, cfl) - 1e-12)
    dt8_stable = B.dg_stable_dt(m8, q8, cfl)
    n8 = n3 * math.ceil(dT / n3 / dt8_stable - 1e-12)
    dt8 = dT / n8
    k8 = m8.field(0.0)
    E, np3 = m3.E, m3.n_p
    data = {}
    for tg in targets:
        rows = snapshots * E * (n3 if tg == "alg1" else 1)
        data[tg] = (torch.empty((rows, 5 * np3), dtype=torch.float32, device="cuda"),
                    torch.empty((rows, 5 * np3), dtype=torch.float32, device="cuda"))
    ref3 = torch.empty((n_eval + 1, 5, E, np3), dtype=torch.float64, device="cuda")
    init = {}
    ws_eq5 = ws_alg1 = None
    _sync()
    t_start = time.perf_counter()
    B.dg_rk_step(m8, q8, k8, dt8, int(round(t0 / dT)) * n8)
    _sync()
    t_ref = time.perf_counter() - t_start
    log(f"P8 reached t0={t0} in {t_ref:.2f}s ({int(round(t0 / dT)) * n8} steps, dt={dt8:.4e})")
    meshes = {P: B.Mesh(N, P, Re) for P in orders}
    for P, m in meshes.items():
        f = m.field()
        B.dg_project(m8, m, q8, f)
        init[P] = f
    B.dg_project(m8, m3, q8, ref3[0])
    t_gen = 0.0
    for j in range(1, n_eval + 1):
        ta = time.perf_counter()
        if j <= snapshots and "alg1" in data:
            X, Y = data["alg1"]
            for i in range(n3):
                r0 = ((j - 1) * n3 + i) * E
                ws_alg1 = B.dg_increment_target(m8, m3, q8, k8, dT / n3, n8 // n3, X[r0:r0 + E], Y[r0:r0 + E],
                                                 ws=ws_alg1)
        else:
            B.dg_rk_step(m8, q8, k8, dt8, n8)
        B.dg_project(m8, m3, q8, ref3[j])
        if j <= snapshots and "eq5" in data:
            X, Y = data["eq5"]
            ws_eq5 = B.dg_forcing_target(m8, m3, q8, X[(j - 1) * E:j * E], Y[(j - 1) * E:j * E], ws=ws_eq5)
        _sync()
        t_gen += time.perf_counter() - ta
    steps8 = n8 * n_eval
    out["reference"] = {"P": 8, "dt": dt8, "steps_to_t0": int(round(t0 / dT)) * n8, "seconds_to_t0": t_ref,
                        "seconds_window_and_eval": t_gen, "steps_window_and_eval": steps8,
                        "wall_per_unit_time_s": t_gen / (eval_end - t0), "low_order_steps_per_snapshot": n3}
    log(f"P8 window + evaluation span: {t_gen:.2f}s, datasets " +
        ", ".join(f"{k} {tuple(v[0].shape)}" for k, v in data.items()))

    # ---------------------------------------------------------------- step 2
    norms = {tg: B.nn_data_stats(X, Y, np3) for tg, (X, Y) in data.items()}
    models = {}
    out["training"] = {"norm": norms, "variants": {}}
    for v in variants:
        X, Y = data[v["target"]]
        rows = X.shape[0]
        nb = rows // batch
        io = MOMENTUM if v["io"] == "momentum" else ALL
        dims = [len(io) * np3] + HIDDEN + [len(io) * np3]
        flops = 3 * 2 * sum(a * b for a, b in zip(dims[:-1], dims[1:])) * batch
        layers = synthetic.mlp_init(dims, seed=seed)
        model = B.Model(dims, B.pack_params(layers), norms[v["target"]], mask=v["mask"], activation=v["act"],
                        in_vars=io, out_vars=io)
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
        models[v["name"]] = (model, v["mode"])
        out["training"]["variants"][v["name"]] = {
            **v, "pairs": rows, "batches_per_epoch": nb, "dims": dims, "seconds": t_train,
            "steps_per_s": v["epochs"] * nb / t_train, "tflops": v["epochs"] * nb * flops / t_train / 1e12,
            "loss_per_epoch": losses}
        log(f"training {v['name']} ({v['target']} pairs, {v['io']}, {v['act']}, {v['mode']}): {v['epochs']} epochs "
            f"x {nb} batches in {t_train:.2f}s, loss {losses[0]:.3e} -> {losses[-1]:.3e}")

    # ---------------------------------------------------------------- step 3
    tmp3 = m3.field()
    err = torch.empty(3, dtype=torch.float64, device="cuda")

    def evolve(mesh, q0, model=None, mode="stage"):
        q = q0.clone()
        k = mesh.field(0.0)
        n = n3 if mesh.P == 3 else math.ceil(dT / B.dg_stable_dt(mesh, q, cfl) - 1e-12)
        dt = dT / n
        step = B.dg_rk_step_post if mode == "post" else B.dg_rk_step
        errs = []
        wall = 0.0
        for j in range(n_eval + 1):
            if j > 0:
                _sync()
                ta = time.perf_counter()
                step(mesh, q, k, dt, n, model=model)
                _sync()
                wall += time.perf_counter() - ta
            if mesh.P == 3:
                B.dg_error_inf(mesh, q, ref3[j], err)
            else:
                B.dg_project(mesh, m3, q, tmp3)
                B.dg_error_inf(m3, tmp3, ref3[j], err)
            errs.append(err.cpu().numpy().tolist())
        e = np.array(errs)
        times = t0 + dT * np.arange(n_eval + 1)
        win = (times > t0) & (times <= t0 + window + 1e-9)
        beyond = times > t0 + window + 1e-9
        return {"P": mesh.P, "mode": mode if model is not None else None, "dt": dt, "steps": n * n_eval,
                "wall_s": wall, "wall_per_unit_time_s": wall / (eval_end - t0),
                "dof_updates_per_s": mesh.E * mesh.n_p * 3 * n * n_eval / wall,
                "e_max_momentum": e.max(axis=1).tolist(), "times": times.tolist(),
                "mean_e_window": float(e[win].max(axis=1).mean()),
                "mean_e_beyond": float(e[beyond].max(axis=1).mean()) if beyond.any() else None,
                "final_e": float(e[-1].max())}

    runs = {}
    runs["P3"] = evolve(m3, ref3[0])
    for name, (model, mode) in models.items():
        runs[f"P3+{name}"] = evolve(m3, ref3[0], model, mode)
    for P in orders:
        runs[f"P{P}"] = evolve(meshes[P], init[P])
    out["runs"] = runs
    for name, r in runs.items():
        log(f"{name:8s} dt={r['dt']:.3e} wall/unit time={r['wall_per_unit_time_s']:.3f}s "
            f"mean e window={r['mean_e_window']:.3e} beyond={r['mean_e_beyond']} final={r['final_e']:.3e}")
    p3 = runs["P3"]
    out["gain"], out["comparison"] = {}, {}
    for name in models:
        p3nn = runs[f"P3+{name}"]
        e3, en = np.array(p3["e_max_momentum"]), np.array(p3nn["e_max_momentum"])
        worse = np.nonzero(en[1:] > e3[1:])[0]
        out["gain"][name] = {"window_ratio": p3nn["mean_e_window"] / p3["mean_e_window"],
                             "beyond_ratio": (p3nn["mean_e_beyond"] / p3["mean_e_beyond"]) if p3["mean_e_beyond"] else None,
                             "better_than_p3_until": p3["times"][1 + worse[0]] if len(worse) else p3["times"][-1]}
        cmp = {}
        for P in orders:
            r = runs[f"P{P}"]
            cmp[f"P{P}"] = {"wall_ratio_vs_p3nn": r["wall_s"] / p3nn["wall_s"],
                            "error_ratio_p3nn_vs_window": p3nn["mean_e_window"] / r["mean_e_window"],
                            "error_ratio_p3nn_vs": p3nn["mean_e_beyond"] / r["mean_e_beyond"] if r["mean_e_beyond"] else None}
        out["comparison"][name] = cmp
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=16)
    ap.add_argument("--Re", type=float, default=1600.0)
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
    a = ap.parse_args()
    variants = None
    if a.variants:
        variants = []
        for item in a.variants.split(";"):
            name, target, io, act, mode, ep, lr = item.split(":")
            variants.append(variant(name, target, io, act, mode, int(ep), float(lr)))
    torch.cuda.set_device(0)
    res = run_study(N=a.N, Re=a.Re, t0=a.t0, window=a.window, snapshots=a.snapshots, eval_end=a.eval_end,
                    epochs=a.epochs, batch=a.batch, lr=a.lr, orders=tuple(int(x) for x in a.orders.split(",")),
                    log=lambda *x: print("[study]", *x, flush=True), variants=variants)
    s = json.dumps(res)
    if a.out:
        open(a.out, "w").write(s)
    print(json.dumps({"gain": res["gain"], "comparison": res["comparison"]}))


if __name__ == "__main__":
    main()
