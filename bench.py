#!/usr/bin/env python3
"""Throughput of the corrected DGSEM hot path on one MI355X.

Headline (``value``): DOF-updates per second per Runge-Kutta stage of the
plain P = 6 Taylor-Green solve, Re 1600, Mach 0.1, 16^3 elements, BR1 viscous
fluxes, FP64, K timed RK3 steps (a step = three stages, each the BR1 gradient
pass and the residual + stage update).  DOF = E (P+1)^3 nodes; every stage
updates every DOF once.

Beside it, on the same JSON line: the corrected P = 3 solve with the forcing
network at every stage (16^3, Re 200), P = 8, the Smagorinsky variants, the
roofline of the dominant kernel (residual + stage update) at P = 6 and at
P = 8 from HIP events around its launches over the same number of steps as
the timed region, with the HBM bytes of the committed rocprofv3 counter
summaries, the mixed Taylor-Green request stream served in real time (p50 /
p99 solve latency), the trained P = 3 + network against plain P = 6 at equal
accuracy beside the paper's figure, and the FP64 CPU oracle timed on the
host (all threads and one thread, plain P = 6 and the corrected P = 3 stage).

    python bench.py [--gpus 1] [--steps 100] [--warmup 1]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALG_BYTES_RESID = 160.0      # read + write q and k per node, one stage update


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the mixed stream replayed for the latency measurement (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-study", action="store_true",
                    help="skip the accuracy-time comparison (trained P=3+NN vs plain P=6 on the 8^3 mesh)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="short run for rocprofv3 counter passes: a 1 GiB device copy, then 5 steps of each workload")
    return ap.parse_args()


def time_steps(B, torch, mesh, q, k, dt, steps, model=None, post=False):
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    step = B.dg_rk_step_post if post else B.dg_rk_step
    t0 = time.perf_counter()
    start.record()
    step(mesh, q, k, dt, steps, model=model)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, start.elapsed_time(stop) / 1e3


def solve_case(B, torch, N, P, Re, Cs, steps, warmup, model=None, post=False, settle_s=0.0):
    mesh = B.Mesh(N, P, Re, Cs=Cs)
    q = mesh.field()
    B.dg_init_tgv(mesh, q)
    dt = B.dg_stable_dt(mesh, q)
    k = mesh.field(0.0)
    if warmup:
        (B.dg_rk_step_post if post else B.dg_rk_step)(mesh, q, k, dt, warmup, model=model)
    if settle_s > 0.0:
        # untimed stepping until the GPU's clocks have settled under this
        # workload: right after start-up a 20-step region otherwise reads
        # up to 8 % slow
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < settle_s:
            B.dg_rk_step(mesh, q, k, dt, 10, model=model)
            torch.cuda.synchronize()
    wall, ev = time_steps(B, torch, mesh, q, k, dt, steps, model, post)
    # the same launches over as many steps, each bracketed by HIP events on
    # the launch stream: mean duration of one launch of each stage kernel
    prof = B.dg_profile_steps(mesh, q, k, dt, steps, model=model)
    nodes = mesh.E * mesh.n_p
    rate = nodes * 3 * steps / wall
    d = B.dg_diagnostics(mesh, q).cpu().numpy()
    return {"N": N, "P": P, "Re": Re, "Cs": Cs, "nodes": nodes, "dt": dt, "steps": steps, "wall_s": wall,
            "event_s": ev, "dof_updates_per_s": rate, "ms_per_step": 1e3 * wall / steps,
            "kernel_ms": prof, "ke_end": float(d[0]), "finite": bool(math.isfinite(d[0]))}


# untimed stepping of the first workload after its warm-up steps, in seconds,
# so that its timed steps start with the GPU's clocks settled
SETTLE_S = 0.3

NET_NORM = [1.0, 0.0, 0.0, 0.0, None, 0.01, 1, 1, 1, 1, 0, 0, 0, 0, 0, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3]


def network_share(k_nn, k_plain):
    """Network share of the corrected stage's kernel time (see the bench
    line's network_share_what)."""
    if k_nn["grad"] == 0.0:
        net = k_nn["net"] - k_plain["grad"]
        return net / max(1e-12, k_nn["net"] + k_nn["resid"])
    return k_nn["net"] / max(1e-12, k_nn["grad"] + k_nn["net"] + k_nn["resid"])


def net_model(B, synthetic, momentum=False, train=False):
    """The Gaussian-initialised forcing network: 320-256-256-256-320 tanh on
    all five variables, or (momentum=True) the paper's form, 192-256-256-256-192
    relu on the three momenta."""
    norm = list(NET_NORM)
    norm[4] = synthetic.TGV_ENERGY_LEVEL
    if momentum:
        dims = [192, 256, 256, 256, 192]
        return B.Model(dims, B.pack_params(synthetic.mlp_init(dims, seed=0)), norm, activation="relu", train=train,
                       in_vars=(1, 2, 3), out_vars=(1, 2, 3))
    dims = [320, 256, 256, 256, 320]
    return B.Model(dims, B.pack_params(synthetic.mlp_init(dims, seed=0)), norm, train=train)


def train_case(B, torch, synthetic, batch, steps, warmup):
    """Adam steps of the 320-256-256-256-320 network on batches of `batch`
    rows drawn from a 16-batch synthetic dataset of TGV-magnitude rows."""
    import numpy as np
    rows = 16 * batch
    x = synthetic.random_rows(rows, 320, seed=5)
    x[:, :64] = 1.0 + 0.01 * x[:, :64]
    x[:, 256:] = synthetic.TGV_ENERGY_LEVEL + x[:, 256:]
    y = synthetic.random_rows(rows, 320, seed=6, scale=1e-3)
    X, Y = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    model = net_model(B, synthetic, train=True)
    idx = torch.from_numpy(np.random.default_rng(0).permutation(rows).astype(np.int32)).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def run(n, first):
        for i in range(n):
            j = (first + i) % 16
            B.nn_train_step(model, X, Y, lr=1e-3, loss=loss, idx=idx[j * batch:(j + 1) * batch])

    run(warmup, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps, warmup)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dims = [320, 256, 256, 256, 320]
    flop = 3 * 2 * sum(a * b for a, b in zip(dims[:-1], dims[1:])) * batch
    return {"batch": batch, "steps": steps, "ms_per_step": 1e3 * wall / steps, "steps_per_s": steps / wall,
            "tflops": flop * steps / wall / 1e12, "gflop_per_step": flop / 1e9,
            "workload": "Adam step, 320-256-256-256-320 tanh, bf16 matrix cores, float32 master weights"}


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    pos = (len(xs) - 1) * p / 100.0
    lo, hi = int(math.floor(pos)), int(math.ceil(pos))
    return xs[lo] + (xs[hi] - xs[lo]) * (pos - lo)


def serving_sample(B, torch, synthetic, n_req):
    """Replays the first n_req requests of the mixed stream (Poisson arrivals,
    mean gap 0.5 s, seed 1; Re, order, mesh drawn uniformly; t_end = 2) in real
    time against the continuous-batching server."""
    reqs = synthetic.request_stream(64, seed=1)[:n_req]
    model = net_model(B, synthetic)
    free = torch.cuda.mem_get_info()[0]
    arena = int(min(free * 0.6, 64 << 30)) & ~255
    srv = B.Server(arena, max_slots=64)
    t0 = time.perf_counter()
    ids = []
    for i, r in enumerate(reqs):
        while time.perf_counter() - t0 < r["arrival"] - reqs[0]["arrival"]:
            time.sleep(0.002)
        ids.append(srv.submit(Re=r["Re"], P=r["P"], N=r["N"], t_end=r["t_end"], use_nn=r["use_nn"],
                              model=model if r["use_nn"] else None, ke_every=50))
        if i % 8 == 7:
            log(f"serving: submitted {i + 1}/{len(reqs)} at {time.perf_counter() - t0:.1f} s")
    last = time.perf_counter()
    while True:
        done = sum(1 for rid in ids if srv.poll(rid)[1].state in (B.SOLVE_DONE, B.SOLVE_FAILED))
        if done == len(ids):
            break
        if time.perf_counter() - last > 10.0:
            log(f"serving: {done}/{len(ids)} solves finished at {time.perf_counter() - t0:.1f} s")
            last = time.perf_counter()
        time.sleep(0.01)
    t_all = time.perf_counter() - t0
    lat, dofs, failed, fallbacks = [], 0, 0, 0
    for rid in ids:
        rc, st = srv.poll(rid)
        if st.state != B.SOLVE_DONE:
            failed += 1
            continue
        fallbacks += st.fallback
        lat.append(st.latency_s)
        dofs += st.dof_updates
    busy, batches = srv.stats()
    srv.close()
    return {"requests": len(reqs), "failed": failed, "fell_back_uncorrected": fallbacks,
            "p50_latency_s": percentile(lat, 50),
            "p99_latency_s": percentile(lat, 99), "makespan_s": t_all, "dof_updates_per_s": dofs / t_all,
            "solves_per_s": len(lat) / t_all, "gpu_busy_fraction": busy / t_all, "step_rounds": batches,
            "stream": "%d of the 64 requests, seed 1, mean gap 0.5 s, Re in {30,200,1600}, "
                      "P in {3+NN,6,8}, N in {4,8,16}, t_end 2" % len(reqs)}


def cpu_baseline(steps=2):
    """The FP64 NumPy oracle on the headline workload (16^3, P = 6, Re 1600
    TGV): `steps` full RK3 steps on all host threads; one stage on a single
    thread; one corrected stage of the 16^3, P = 3, Re 200 workload (residual
    plus the float64 network) on all threads."""
    import numpy as np
    import synthetic
    from oracle import dg, forcing, mlp, rk
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    prm = dg.Params(N=16, P=6, Re=1600.0)
    q = dg.tgv_initial_condition(prm)
    dt = dg.stable_dt(q, prm)
    nodes = q[0].size
    t0 = time.perf_counter()
    rk.integrate(q, dt, steps, lambda qq, t: dg.residual(qq, prm))
    t_all = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        dg.residual(q, prm)
        t_one = time.perf_counter() - t0
    prm3 = dg.Params(N=16, P=3, Re=200.0)
    q3 = dg.tgv_initial_condition(prm3)
    dims = [320, 256, 256, 256, 320]
    params = [(mlp.bf16_round(W), b.astype(np.float64)) for W, b in synthetic.mlp_init(dims, seed=0)]
    nrm = list(NET_NORM)
    nrm[4] = synthetic.TGV_ENERGY_LEVEL
    norm = forcing.Normalisation(nrm[0:5], nrm[5:10], nrm[10:15], nrm[15:20])
    t0 = time.perf_counter()
    forcing.corrected_rhs(q3, prm3, params, norm)
    t_c3 = time.perf_counter() - t0
    return {"value": nodes * 3 * steps / t_all, "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} full RK3 steps ({3 * steps} residuals) of the 16^3 P=6 Re-1600 TGV, "
                      f"NumPy float64, {t_all:.1f} s on {threads} threads",
            "host_cpus": os.cpu_count(),
            "single_thread": {"value": nodes / t_one, "unit": "DOF-updates/s", "cores": 1,
                              "sample": f"one residual (one stage) of the same workload, {t_one:.1f} s"},
            "corrected_p3_stage": {"value": q3[0].size / t_c3, "unit": "DOF-updates/s", "cores": threads,
                                   "sample": "one corrected stage (residual + float64 320-256-256-256-320 "
                                             f"network) of the 16^3 P=3 Re-200 TGV, {t_c3:.2f} s"}}


def counter_traffic(kernel_file, tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{tag}_counters.md")
    if not os.path.exists(path):
        return None
    src = open(os.path.join(ROOT, "paper_2207_11571_amd", "csrc", kernel_file), "rb").read()
    sha = hashlib.sha256(src).hexdigest()[:16]
    rec = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            key, val = line[2:].split(":", 1)
            rec[key.strip()] = val.strip()
    if rec.get("source_sha256_16") != sha:
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs one solve on one GPU: --gpus must be 1 "
                                   "(sharding a solve over several GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    import synthetic
    from paper_2207_11571_amd import binding as B
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    B.lib()

    if args.profile_pass:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        for (P, Re, Cs) in ((6, 1600.0, 0.0), (8, 1600.0, 0.0)):
            solve_case(B, torch, 16, P, Re, Cs, 5, 0)
        solve_case(B, torch, 16, 3, 200.0, 0.0, 5, 0, model=net_model(B, synthetic))
        # the correction after each step (Algorithm 1): at 16^3 the network
        # runs fused with the first stage's BR1 pass
        solve_case(B, torch, 16, 3, 200.0, 0.0, 5, 0, model=net_model(B, synthetic, momentum=True), post=True)
        # the stand-alone network launch (the server's batched solves, meshes
        # too small for the fused launch) on the 16^3 state
        m = B.Mesh(16, 3, 200.0)
        q = m.field()
        B.dg_init_tgv(m, q)
        s = m.field(0.0)
        model = net_model(B, synthetic)
        for _ in range(5):
            B.nn_forcing(model, m, q, s)
        torch.cuda.synchronize()
        log("profile pass done")
        return

    log("P6 headline")
    head = solve_case(B, torch, 16, 6, 1600.0, 0.0, args.steps, args.warmup, settle_s=SETTLE_S)
    log("P8")
    p8 = solve_case(B, torch, 16, 8, 1600.0, 0.0, args.steps, args.warmup)
    log("LES variants")
    p6les = solve_case(B, torch, 16, 6, 1600.0, 0.1, args.steps, args.warmup)
    p8les = solve_case(B, torch, 16, 8, 1600.0, 0.1, args.steps, args.warmup)
    log("P3 + network")
    model = net_model(B, synthetic)
    p3nn = solve_case(B, torch, 16, 3, 200.0, 0.0, args.steps, args.warmup, model=model)
    p3 = solve_case(B, torch, 16, 3, 200.0, 0.0, args.steps, args.warmup)
    log("P3 + paper-form network after each step (Algorithm 1)")
    p3post = solve_case(B, torch, 16, 3, 200.0, 0.0, args.steps, args.warmup,
                        model=net_model(B, synthetic, momentum=True), post=True)
    log("training step, batch 4096")
    training = train_case(B, torch, synthetic, 4096, 50, 5)

    def resid_roofline(case, kernel, tag):
        ms = case["kernel_ms"]["resid"]
        alg = ALG_BYTES_RESID * case["nodes"]
        achieved = alg / (ms * 1e-3) / 1e9
        traffic = counter_traffic("dg_kernels.hip", tag)
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
                "algorithmic_bytes_per_launch": alg, "mean_launch_ms": ms,
                "traffic_over_algorithmic": None if traffic is None else traffic / alg,
                "counter_GBs": None if traffic is None else traffic / (ms * 1e-3) / 1e9,
                "counter_frac": None if traffic is None else traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "stage_algorithmic_frac": case["dof_updates_per_s"] * ALG_BYTES_RESID / (HBM_PEAK_GBS * 1e9)}

    roofline = resid_roofline(head, "k_resid1<7,1> (residual + RK stage update, 16^3 P=6, one solve: descriptor in the kernel arguments)", "k_resid_p6")
    roofline["p8"] = resid_roofline(p8, "k_resid_loop<9,1> (residual + RK stage update, 16^3 P=8, one block per CU walking the elements)", "k_resid_p8")
    stage_alg_frac = roofline["stage_algorithmic_frac"]

    serving = None
    if args.serve_requests > 0:
        log("serving sample")
        serving = serving_sample(B, torch, synthetic, args.serve_requests)

    study = None
    if not args.no_study:
        log("accuracy-time study (8^3)")
        from paper_2207_11571_amd import study as st
        res = st.run_study(N=8, Re=1600.0, t0=4.0, window=0.15, snapshots=100, eval_end=4.45, batch=512,
                           orders=(5, 6), variants=[st.variant("nn", epochs=200),
                                                    st.variant("alg1", "alg1", "momentum", "relu", "post", epochs=200),
                                                    st.variant("alg1a", "alg1", "all", "tanh", "post", epochs=200)],
                           log=lambda *a: None)
        runs = res["runs"]
        study = {"config": "8^3 elements, Re 1600, P=8 reference from t=0; training pairs every 0.0015 (one P=3 "
                           "step) over [4, 4.15]: 'nn' Eq. (5) pairs, all variables, tanh, forcing every stage; "
                           "'alg1' Algorithm 1 increments, momentum in/out, relu, correction after each step; "
                           "'alg1a' Algorithm 1 increments and correction, all variables, tanh; 200 epochs Adam "
                           "batch 512; evaluation to t=4.45; e_n = max momentum error vs filtered P=8 (Eq. 9) "
                           "on the P=3 space",
                 "training_s": {k: v["seconds"] for k, v in res["training"]["variants"].items()},
                 "reference_p8_s": res["reference"]["seconds_to_t0"] + res["reference"]["seconds_window_and_eval"]}
        for name in ("P3", "P3+nn", "P3+alg1", "P3+alg1a", "P5", "P6"):
            r = runs[name]
            study[name] = {"mean_e_window": r["mean_e_window"], "mean_e_beyond": r["mean_e_beyond"],
                           "wall_per_unit_time_s": r["wall_per_unit_time_s"], "dt": r["dt"]}
        study["p6_wall_over_p3nn"] = {k: runs["P6"]["wall_s"] / runs["P3+" + k]["wall_s"] for k in ("nn", "alg1", "alg1a")}
        study["equal_accuracy_speedup_over_p6"] = {
            "measured": {k: study["p6_wall_over_p3nn"][k] for k in ("nn", "alg1", "alg1a")
                         if runs["P3+" + k]["mean_e_window"] <= runs["P6"]["mean_e_window"]},
            "what": "wall time of plain P=6 over wall time of the trained P=3 + network over the same physical "
                    "time, same mesh and Reynolds number, for the networks whose mean window error e_n is at most "
                    "P=6's",
            "paper": 4.94,
            "paper_what": "Table 2: P=6 cost over P=3 + NN cost, Re 1600, t = 7, 8^3 elements, HORSES3D on one "
                          "Intel Core i7 at 3.07 GHz (Sec. 2.6)"}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline()

    out = {
        "metric": "DOF-updates/s per RK stage (P=3+NN vs plain P=6) and p50/p99 solve latency",
        "value": head["dof_updates_per_s"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (analytic Taylor-Green initial state; Gaussian-initialised network, seed 0)",
        "config": {"workload": "plain DG, TGV Re 1600 Mach 0.1, 16^3 elements, P=6, BR1, no closure, "
                               "FP64 RK3 (the P=6 half of the throughput configuration)",
                   "N": 16, "P": 6, "Re": 1600, "nodes": head["nodes"], "dt": head["dt"],
                   "untimed_settle_s": SETTLE_S},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stage_algorithmic_hbm_fraction": stage_alg_frac,
        "p3_nn": {"dof_updates_per_s": p3nn["dof_updates_per_s"], "ms_per_step": p3nn["ms_per_step"],
                  "kernel_ms": p3nn["kernel_ms"],
                  "grad_and_network_fused": p3nn["kernel_ms"]["grad"] == 0.0,
                  "network_share_of_stage": network_share(p3nn["kernel_ms"], p3["kernel_ms"]),
                  "network_share_what": "network time over the stage's kernel time; where the BR1 pass and the "
                                        "network run as one launch, the network time is that launch minus the "
                                        "BR1 pass of plain P=3 on the same mesh",
                  "workload": "corrected P=3, 16^3, Re 200, 320-256-256-256-320 tanh bf16 network every stage"},
        "p3_plain": {"dof_updates_per_s": p3["dof_updates_per_s"], "ms_per_step": p3["ms_per_step"]},
        "p3_nn_post": {"dof_updates_per_s": p3post["dof_updates_per_s"], "ms_per_step": p3post["ms_per_step"],
                       "workload": "P=3, 16^3, Re 200, 192-256-256-256-192 relu network on the momenta, "
                                   "correction after each step (Algorithm 1)"},
        "training": training,
        "p8": {"dof_updates_per_s": p8["dof_updates_per_s"], "ms_per_step": p8["ms_per_step"],
               "kernel_ms": p8["kernel_ms"],
               "resid_hbm_alg_GBs": ALG_BYTES_RESID * p8["nodes"] / (p8["kernel_ms"]["resid"] * 1e-3) / 1e9},
        "p6_les": {"dof_updates_per_s": p6les["dof_updates_per_s"]},
        "p8_les": {"dof_updates_per_s": p8les["dof_updates_per_s"]},
        "serving": serving,
        "accuracy_time_8cubed": study,
        "kernel_ms_p6": head["kernel_ms"],
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
