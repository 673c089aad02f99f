"""Benchmark of the reduced-KKT hot path on one MI355X.

One step = one pass of the whole per-iteration hot path over all scenarios:
evaluate (f, g, h, Jacobians, Hessian of the Lagrangian), condense (K, LU of
G_x, local reduction, scenario sum), factor (dense Cholesky) and step
(reduced right-hand side, p_u, recovery), through the C ABI, on a seeded
synthetic iterate whose inputs are resident in device memory.

Printed JSON line: the whole-path throughput in scenario-IPM-iterations/s,
the condense+factor throughput next to the same kernels launched one
scenario at a time (the plain per-scenario form), the roofline position of
the dominant stage (HIP events on the launch stream inside the timed
region) and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--config c1|c4] [--no-cpu] [--no-plain]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6           # MI355X FP64 vector (and FP64 matrix) TFLOP/s

WORKLOADS = {
    "warm": "learned warm start on the 118-bus grid (load draws sigma 0.15)",
    "c1": "118-bus / 186-line / 54-generator synthetic grid (the sizes of the paper's case118), "
          "N = 128 load scenarios (sigma 0.1), n_x = 181, n_u = 107; full hot path per step",
    "c4": "9241-bus / 16049-line / 1445-generator synthetic grid (the sizes of the paper's "
          "case9241pegase), N = 16 load scenarios (sigma 0.1), n_x = 17036, n_u = 2889; full hot path per step",
    "c2": "64 independent single-scenario grids, n_bus log-uniform in [300, 2000], 1.5 n_bus lines, "
          "0.15 n_bus generators; launch shapes autotuned per instance; one multi-instance pass (one launch "
          "per kernel configuration, captured as one graph) vs the 64 passes one after the other",
}


def warm_main(args):
    """Learned warm start on the 118-bus grid: cold device IPM solves of
    seeded load draws (sigma 0.15), the perceptron 198 -> 512 -> 512 -> 512
    -> 896 trained on the first n_train, warm solves of the rest."""
    import torch
    import synthgrid as sg
    from paper_2301_04869_amd import warmstart as ws
    n_tr, n_va, n_te = args.n_train, args.n_val, args.n_test
    inst = sg.preset("c3", n_scen=n_tr + n_va + n_te)
    res = ws.experiment(torch, inst.net, inst.scen.pd, inst.scen.qd, n_train=n_tr, n_val=n_va,
                        mu0s=(1e-4, 1e-5, 1e-6, 1e-7, 1e-8), steps=args.train_steps,
                        log=lambda m: print(m, file=sys.stderr, flush=True))
    # training-step rate of the perceptron alone (batch 256), HIP events
    dd = sg.dims(inst.net.n_bus, inst.net.n_line, inst.net.n_gen)
    sizes = [2 * len(inst.net.load_bus), 512, 512, 512, 2 * dd["n_x"] + dd["n_u"] + dd["m"]]
    import paper_2301_04869_amd as R
    m = R.Mlp(sizes, 256)
    m.set_params(torch.tensor(ws.init_params(sizes, 0), device="cuda"))
    x = torch.randn(256, sizes[0], device="cuda")
    t = torch.randn(256, sizes[-1], device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for _ in range(20):
        m.train_step(x, t, 1e-4, loss)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(200):
        m.train_step(x, t, 1e-4, loss)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / 200
    n_par = m.n_params
    flops = 6.0 * 256 * sum(a * b for a, b in zip(sizes[:-1], sizes[1:]))
    out = {"metric": "mean IPM iterations per solve, cold vs learned warm start (fallbacks counted)",
           "value": res["warm_mean_iters"], "unit": "IPM iterations", "n_gpus": 1,
           "steps": res["n_test"], "warmup": 0, "ms_per_step": None, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64 solves, bf16 products in the MLP",
           "data": "synthetic",
           "config": {"workload": "118-bus grid, load draws sigma 0.15 (the warm-start set); MLP "
                      f"{sizes}, {n_par} parameters; {n_tr} training / {n_va} validation / {n_te} "
                      "test draws; warm-start mu0 chosen on the validation draws",
                      "train_steps": args.train_steps, "mu0_warm": res["mu0_warm"],
                      "validation_mean_iters": res["validation_mean_iters"]},
           "cold_mean_iters": res["cold_mean_iters"], "fallback_rate": res["fallback_rate"],
           "mean_start_mean_iters": res["mean_start_mean_iters"],
           "mean_start_fallback_rate": res["mean_start_fallback_rate"],
           "max_rel_obj_diff": res["max_rel_obj_diff"], "cold_solve_seconds": res["cold_solve_seconds"],
           "train_seconds": res["train_seconds"],
           "mlp_train_step_ms": step_ms, "mlp_samples_per_s": 256 / (step_ms * 1e-3),
           "mlp_roofline": {"bound": "mfma", "achieved": flops / (step_ms * 1e-3) / 1e12, "peak": 2500.0,
                            "unit": "TFLOP/s", "frac": flops / (step_ms * 1e-3) / 1e12 / 2500.0,
                            "traffic": None}}
    print(json.dumps(out), flush=True)


def multi_main(args):
    """64 independent single-scenario grids of uneven size (n_bus log-uniform
    in [300, 2000]) in one multi-instance handle: every kernel of the pass
    launched once per configuration group for all instances (eager and as one
    captured graph), against the 64 instances' own passes run one after the
    other.  Launch shapes from the autotuner, per instance."""
    import torch
    import synthgrid as sg
    from synthgrid.iterates import random_iterate
    import paper_2301_04869_amd as R
    insts = sg.batch_instances(64, seed=2000)
    zf = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda")  # noqa: E731
    handles, arglist, shapes = [], [], []
    t0 = time.time()
    for j, inst in enumerate(insts):
        pd, qd = inst.scen.pd.T, inst.scen.qd.T
        best = R.rkkt_autotune(inst.net, pd, qd, reps=2)[0] if args.autotune else {}
        p = R.rkkt_create(inst.net, pd, qd, **best)
        d = p.dims
        nx, nu, m = d["n_x"], d["n_u"], d["m"]
        it = random_iterate(inst.net, 1, 3000 + j)
        t = {k: torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device="cuda")
             for k, v in it.items() if k != "obj_weight"}
        a = dict(x=t["x"], u=t["u"], y=t["y"], z=t["z"], obj_weight=it["obj_weight"], f=zf(1), grad_x=zf(1, nx),
                 grad_u=zf(1, nu), g=zf(1, nx), h=zf(1, m), sigma_x=t["sigma_x"], sigma_u=t["sigma_u"],
                 sigma_s=t["sigma_s"], khat=zf(nu, nu), chol=zf(nu, nu),
                 info=torch.zeros(1, dtype=torch.int32, device="cuda"), r1x=t["r1x"], r1u=t["r1u"],
                 r2=t["r2"], r3=t["r3"], r4=t["r4"], px=zf(1, nx), pu=zf(nu), ps=zf(1, m), py=zf(1, nx),
                 pz=zf(1, m))
        R.rkkt_evaluate(p, a["x"], a["u"], a["y"], a["z"], a["obj_weight"], a["f"], a["grad_x"], a["grad_u"],
                        a["g"], a["h"])
        a["delta_w"] = find_delta_w(R, torch, p, t, a["khat"], a["chol"], a["info"])
        handles.append(p)
        arglist.append(a)
        shapes.append({"n_bus": inst.net.n_bus, "n_x": nx, "n_u": nu, "variant": d["variant"],
                       "col_tile": d["col_tile"], "lds_reduce": d["lds_reduce"], "sweep_form": d["sweep_form"],
                       "scen_per_group": d["scen_per_group"], "chain_rows": d["chain_rows"]})
        if (j + 1) % 8 == 0:
            progress(f"{j + 1} of 64 instances set up ({time.time() - t0:.0f} s)")
    setup_s = time.time() - t0
    stream = torch.cuda.current_stream()
    # reference: the instances' own passes, one after the other
    for p, a in zip(handles, arglist):
        R.rkkt_iterate(p, a, stream)
    torch.cuda.synchronize()
    ref = [(a["khat"].clone(), a["pu"].clone(), a["px"].clone()) for a in arglist]
    mh = R.Multi(handles, arglist)
    for a in arglist:
        for k in ("khat", "pu", "px"):
            a[k].fill_(float("nan"))
    mh.iterate(stream)
    torch.cuda.synchronize()
    same = all(torch.equal(a["khat"], r[0]) and torch.equal(a["pu"], r[1]) and torch.equal(a["px"], r[2])
               for a, r in zip(arglist, ref))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn, k):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    def sequential():
        for p, a in zip(handles, arglist):
            R.rkkt_iterate(p, a, stream)

    seq_ms = timed(sequential, max(3, args.steps // 4))
    progress(f"64 sequential passes: {seq_ms:.3f} ms")
    eager_ms = timed(lambda: mh.iterate(stream), args.steps)
    progress(f"multi-instance pass, eager: {eager_ms:.3f} ms")
    mh.capture()
    graph_ms = timed(lambda: mh.launch(stream), args.steps)
    progress(f"multi-instance pass, graph: {graph_ms:.3f} ms")
    torch.cuda.synchronize()
    same = same and all(torch.equal(a["khat"], r[0]) and torch.equal(a["pu"], r[1]) for a, r in zip(arglist, ref))
    ms = min(eager_ms, graph_ms)
    out = {"metric": "instance-IPM-iterations/s, 64 independent instances of uneven size in one "
                     "multi-instance pass vs the 64 passes one after the other",
           "value": 64 / (ms * 1e-3), "unit": "instance-IPM-iterations/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": WORKLOADS["c2"], "instances": len(shapes), "autotuned": bool(args.autotune),
                      "n_bus_min": min(x["n_bus"] for x in shapes), "n_bus_max": max(x["n_bus"] for x in shapes)},
           "graph_ms_per_step": graph_ms, "eager_ms_per_step": eager_ms,
           "launches_per_pass": mh.n_launches,
           "sequential": {"ms_per_iteration": seq_ms, "value": 64 / (seq_ms * 1e-3),
                          "what": "each instance's own rkkt_iterate pass, one after the other"},
           "speedup_vs_sequential": seq_ms / ms, "outputs_equal_to_sequential": bool(same),
           "setup_seconds": setup_s, "shapes": shapes}
    print(json.dumps(out), flush=True)


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_work(d):
    """The method's own work per launch of every stage: (flops, bytes).

    Bytes: every input read once, every value array the method materialises
    (the Jacobian values G_x and G_u, K = W + H^T Sigma_s H, the LU factors,
    the reduced matrix) written once by the stage that makes it and read once
    by each stage that needs it, outputs written once; the shared index
    arrays (patterns, schedules) once per pass, charged to the reduction.
    Flops: the multiply-adds (2 flops each) of the sparse LU, of the
    triangular solves with the n_u right-hand sides and the sparse K and G_u
    products of the paper's adjoint closure (two forward and two adjoint
    solves per column), the condensation products, the scenario sum and the
    Cholesky; no evaluation flops are counted.  Work a launch does beyond
    this (the stacked variant's dense Z^T (K Z) product and its panels of Z
    and K Z in device memory, per-scenario partial matrices) is returned in
    a second dict, "beyond", stage -> (flops, bytes)."""
    N, nx, nu, m = d["n_scen"], d["n_x"], d["n_u"], d["m"]
    nz = nx + nu
    nlu, ngu, ngx, nh = d["nnz_lu"], d["nnz_gu"], d["nnz_gx"], d["nnz_h"]
    kxx, kxu, kuu = d["nnz_kxx"], d["nnz_kxu"], d["nnz_kuu"]
    nload, ntrip, idx = d["n_load"], d["n_trip"], d["idx_bytes"]
    nu_pad = (nu + 63) // 64 * 64      # row pitch of the stacked panels
    w, beyond = {}, {}
    w["evaluate"] = (0.0, 8 * N * (2 * nx + m + 2 * nload) + 8 * nu            # x, y, z, loads; u
                     + 8 * N * (1 + 2 * nx + m + nu)                          # f, g, h, gradients
                     + 8 * N * (ngx + ngu))                                   # G_x, G_u values
    w["condense_values"] = (3.0 * N * ntrip, 8 * N * (nx + m) + 8 * N * (kxx + 2 * kxu + kuu))
    w["refactor"] = (2.0 * N * d["lu_update_flops"], 8 * N * (ngx + nlu))
    if d["variant"] == 2:
        # forward solves and K products; the closure is the stacked product
        w["reduce"] = (2.0 * N * nu * (nlu + kxx + kxu),
                       8 * N * (nlu + kxx + 2 * kxu + kuu + ngu) + idx)
        beyond["reduce"] = (0.0, 8 * N * (nx + nz) * nu_pad)
        w["stacked_product"] = (2.0 * N * nu * (nlu + ngu), 8 * nu * nu)
        beyond["stacked_product"] = (1.0 * N * nz * nu * (nu + 1), 16 * N * nz * nu_pad)
    else:
        w["reduce"] = (2.0 * N * nu * (2 * nlu + kxx + kxu + ngu),
                       8 * N * (nlu + kxx + 2 * kxu + kuu + ngu) + idx)
        beyond["reduce"] = (0.0, 8 * N * nu * nu)
    w["scenario_sum"] = (1.0 * N * nu * nu, 8 * nu * nu + 8 * nu)
    w["factor"] = (nu ** 3 / 3.0, 16 * nu * nu)
    # reduced right-hand side: H^T w, adjoint solve of r1_hat, forward solve of
    # r3, K_xx q and its adjoint solve, G_u^T and K_ux products
    w["step_rhs"] = (2.0 * N * (3 * nlu + nh + kxx + kxu + 2 * ngu),
                     8 * N * (2 * nx + 3 * m) + 8 * N * (nlu + kxx + kxu + nh + ngu) + 8 * N * nu)
    w["reduced_solve"] = (2.0 * nu * nu + N * nu, 8 * (nu * nu + N * nu + 2 * nu))
    # p_x (forward solve), p_y (adjoint solve), H p_d, p_s, p_z
    w["step_recover"] = (2.0 * N * (2 * nlu + ngu + kxx + kxu + 2 * nh),
                         8 * N * (2 * nx + 3 * m) + 8 * N * (nlu + kxx + kxu + nh + ngu)
                         + 8 * N * (2 * nx + 2 * m))
    return w, beyond


def method_totals(d):
    """Per-iteration totals of the method's work as the scope table defines
    them for condense + factor: F = N [F_LU + n_u (4 nnz_LU + 2 nnz_Kxx +
    2 nnz_Kxu + 2 nnz_Gu)] + N n_u^2 + n_u^3 / 3 and B = 8 N [(3 n_x + 2 m +
    2 n_load) + 2 (nnz_Gx + nnz_Gu + nnz_Kxx + nnz_Kxu + nnz_LU)] + idx +
    24 n_u^2."""
    N, nx, nu, m = d["n_scen"], d["n_x"], d["n_u"], d["m"]
    nlu, ngu, ngx = d["nnz_lu"], d["nnz_gu"], d["nnz_gx"]
    kxx, kxu = d["nnz_kxx"], d["nnz_kxu"]
    F = N * (2.0 * d["lu_update_flops"] + nu * (4 * nlu + 2 * kxx + 2 * kxu + 2 * ngu)) \
        + N * nu * nu + nu ** 3 / 3.0
    B = 8.0 * N * ((3 * nx + 2 * m + 2 * d["n_load"]) + 2 * (ngx + ngu + kxx + kxu + nlu)) \
        + d["idx_bytes"] + 24.0 * nu * nu
    return F, B


def roof_time(flops, nbytes):
    """Time at the roofline: max(bytes / HBM peak, flops / FP64 peak), s."""
    return max(nbytes / (HBM_PEAK_GBS * 1e9), flops / (FP64_PEAK_TFS * 1e12))


def measured_traffic(stage, workload):
    """HBM bytes per launch of `stage` from the committed counter record
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when there is
    none for this stage and workload or the kernel's source changed since."""
    root = os.path.dirname(os.path.abspath(__file__))
    if not os.path.isdir(os.path.join(root, "profiles")):
        return None
    for name in sorted(os.listdir(os.path.join(root, "profiles"))):
        if not (name.startswith("hbm_traffic_") and name.endswith(".json")):
            continue
        with open(os.path.join(root, "profiles", name)) as fh:
            rec = json.load(fh)
        if rec.get("stage") != stage or rec.get("workload") != workload:
            continue
        with open(os.path.join(root, rec["source"]), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != rec["source_sha256"]:
                return None
        return rec["bytes_per_launch"]
    return None


def roofline_entry(stage, ms, count, d, workload):
    work, beyond = stage_work(d)
    flops, nbytes = work[stage]
    traffic = measured_traffic(stage, workload)
    t = ms / count * 1e-3
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (FP64_PEAK_TFS * 1e12)
    extra = {"kernel_stage": stage, "avg_ms": ms / count, "algorithmic_bytes": nbytes,
             "algorithmic_flops": flops}
    if stage in beyond:
        extra["beyond_algorithmic"] = {"flops": beyond[stage][0], "bytes": beyond[stage][1]}
    if t_hbm >= t_alu:
        ach = nbytes / t / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": traffic, **extra}
    ach = flops / t / 1e12
    return {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
            "frac": ach / FP64_PEAK_TFS, "traffic": traffic, **extra}


def pass_roofline(d, ms_per_step, cf_ms):
    """Whole-pass and condense+factor fractions: roofline time of the method's
    work over the measured time."""
    work, _ = stage_work(d)
    fl = sum(v[0] for v in work.values())
    by = sum(v[1] for v in work.values())
    t_pass = roof_time(fl, by)
    F, B = method_totals(d)
    t_cf = roof_time(F, B)
    return {"pass": {"flops": fl, "bytes": by, "roof_us": t_pass * 1e6, "measured_us": ms_per_step * 1e3,
                     "frac": t_pass / (ms_per_step * 1e-3)},
            "condense_factor": {"flops": F, "bytes": B, "roof_us": t_cf * 1e6,
                                "measured_us": cf_ms * 1e3, "frac": t_cf / (cf_ms * 1e-3)}}


def attach_probe_peaks(out, probe):
    """The rates the copy and FP64 probes reach on this device, and the
    roofline fractions against them beside those against the datasheet peaks
    (HBM 8 TB/s; FP64 vector and matrix core 78.6 TFLOP/s)."""
    out["probe_peaks"] = {"hbm_gbs": probe["hbm_gbs"], "fp64_vec_tfs": probe["fp64_vec_tfs"],
                          "fp64_mfma_tfs": probe["fp64_mfma_tfs"],
                          "what": "1 GiB device copy; 8 independent FP64 FMA chains per thread; "
                                  "4 independent v_mfma_f64_16x16x4f64 accumulations per wavefront"}
    roof = out["roofline"]
    meas = probe["hbm_gbs"] if roof["bound"] == "hbm" else probe["fp64_vec_tfs"]
    roof["measured_peak"] = meas
    roof["frac_of_measured"] = roof["achieved"] / meas
    for part in out["roofline_pass"].values():
        t = max(part["bytes"] / (probe["hbm_gbs"] * 1e9), part["flops"] / (probe["fp64_vec_tfs"] * 1e12))
        part["roof_us_measured_peaks"] = t * 1e6
        part["frac_of_measured"] = t / (part["measured_us"] * 1e-6)


def find_delta_w(R, torch, p, t, khat, chol, info):
    """Inertia correction of the interior-point rules: delta_w = 0, then 1e-4,
    x100 until the reduced matrix factorises."""
    dw = 0.0
    while True:
        R.rkkt_condense(p, t["sigma_x"], t["sigma_u"], t["sigma_s"], dw, khat)
        chol.copy_(khat)
        R.rkkt_factor(p, chol, info)
        torch.cuda.synchronize()
        if int(info.item()) == 0:
            return dw
        dw = 1e-4 if dw == 0.0 else 100.0 * dw
        if dw > 1e20:
            raise RuntimeError("inertia correction failed")


def cpu_baseline(inst, it, dw, budget_s=12.0):
    """The oracle (as it stands) on the same iterate: evaluation, diagonals,
    reduced matrix, Cholesky and Newton step for a bounded number of
    scenarios, repeated until the time budget is used."""
    from threadpoolctl import threadpool_limits
    import synthgrid as sg
    from oracle import kkt
    cores = len(os.sched_getaffinity(0))
    net, N = inst.net, inst.scen.n_scen
    ns = min(N, 16 if net.n_bus > 1000 else 32)
    sub = sg.Instance(inst.name, net, sg.Scenarios(inst.scen.pd[:, :ns], inst.scen.qd[:, :ns],
                                                   inst.scen.sigma, inst.scen.seed))
    prob = kkt.Problem(sub)
    z = np.zeros
    I = kkt.Iterate(it["x"][:ns], it["u"], z((ns, prob.m)), it["y"][:ns], it["z"][:ns],
                    z((ns, prob.n_x)), z((ns, prob.n_x)), z(prob.n_u), z(prob.n_u), z((ns, prob.m)),
                    z((ns, prob.m)))
    dg = kkt.Diag(it["sigma_x"][:ns], it["sigma_u"], it["sigma_s"][:ns])
    rs = kkt.Resid(it["r1x"][:ns], it["r1u"], it["r2"][:ns], it["r3"][:ns], it["r4"][:ns])

    def timed(threads, nsub, budget):
        sp = prob if nsub == ns else kkt.Problem(sg.Instance(
            inst.name, net, sg.Scenarios(inst.scen.pd[:, :nsub], inst.scen.qd[:, :nsub], inst.scen.sigma,
                                         inst.scen.seed)))
        Ii = kkt.Iterate(**{k: (a[:nsub] if a.ndim == 2 else a) for k, a in I.__dict__.items()})
        dgi = kkt.Diag(dg.sx[:nsub], dg.su, dg.ss[:nsub])
        rsi = kkt.Resid(rs.r1x[:nsub], rs.r1u, rs.r2[:nsub], rs.r3[:nsub], rs.r4[:nsub])
        passes = 0
        t0 = time.perf_counter()
        with threadpool_limits(limits=threads):
            while True:
                ev = kkt.evaluate(sp, Ii, it["obj_weight"])
                red = kkt.reduced_hessian(sp, ev, dgi, dw)
                kkt.newton_reduced(sp, ev, dgi, rsi, dw, red)
                passes += 1
                el = time.perf_counter() - t0
                if el >= budget or (net.n_bus > 1000 and passes >= 1):
                    break
        return nsub * passes / el, passes, el

    v, passes, el = timed(cores, ns, budget_s)
    progress(f"oracle on {cores} threads: {v:.3g} scenario-IPM-iterations/s")
    # the same oracle on one host thread, on a smaller sample
    n1 = 1 if net.n_bus > 1000 else 8
    v1, p1, el1 = timed(1, n1, budget_s / 2)
    return {"value": v, "unit": "scenario-IPM-iterations/s", "cores": cores, "kind": "oracle",
            "sample": f"{passes} pass(es) of evaluate + reduced matrix + Cholesky + Newton step over "
                      f"{ns} of the {N} scenarios, {el:.1f} s, BLAS threads = {cores}",
            "single_thread": {"value": v1, "unit": "scenario-IPM-iterations/s", "cores": 1,
                              "sample": f"{p1} pass(es) over {n1} scenario(s), {el1:.1f} s, "
                                        "BLAS threads = 1"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--col-tile", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0, choices=(0, 1, 2),
                    help="reduction: 1 adjoint solves, 2 stacked product, 0 automatic")
    ap.add_argument("--sweep-form", type=int, default=0, choices=(0, 1, 2),
                    help="reduction solve schedules: 1 push, 2 pull, 0 automatic")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="c2: automatic launch shapes instead of the autotuner's")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the copy / FP64 probes of the machine balance")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--n-train", type=int, default=20000, help="warm: training draws")
    ap.add_argument("--n-val", type=int, default=200, help="warm: validation draws (choice of mu0)")
    ap.add_argument("--n-test", type=int, default=2000, help="warm: held-out draws")
    ap.add_argument("--train-steps", type=int, default=20000, help="warm: Adam steps")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device copies of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the scenario split across GPUs is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8, "copies": 5}))
        return
    import synthgrid as sg
    from synthgrid.iterates import random_iterate
    import paper_2301_04869_amd as R

    R.lib()
    if args.config == "c2":
        multi_main(args)
        return
    if args.config == "warm":
        warm_main(args)
        return
    inst = sg.preset(args.config)
    net, N = inst.net, inst.scen.n_scen
    it = random_iterate(net, N, args.seed)
    p = R.rkkt_create(net, inst.scen.pd.T, inst.scen.qd.T, col_tile=args.col_tile,
                      variant=args.variant, sweep_form=args.sweep_form)
    d = p.dims
    nx, nu, m = d["n_x"], d["n_u"], d["m"]
    t = {k: torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device="cuda")
         for k, v in it.items() if k != "obj_weight"}
    w = it["obj_weight"]
    zf = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda")  # noqa: E731
    f, gx, gu, g, h = zf(N), zf(N, nx), zf(N, nu), zf(N, nx), zf(N, m)
    khat, chol = zf(nu, nu), zf(nu, nu)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    px, pu, ps, py, pz = zf(N, nx), zf(nu), zf(N, m), zf(N, nx), zf(N, m)
    stream = torch.cuda.current_stream()

    R.rkkt_evaluate(p, t["x"], t["u"], t["y"], t["z"], w, f, gx, gu, g, h)
    dw = find_delta_w(R, torch, p, t, khat, chol, info)

    def step():
        R.rkkt_evaluate(p, t["x"], t["u"], t["y"], t["z"], w, f, gx, gu, g, h, stream)
        R.rkkt_condense(p, t["sigma_x"], t["sigma_u"], t["sigma_s"], dw, khat, stream)
        chol.copy_(khat)
        R.rkkt_factor(p, chol, info, stream)
        R.rkkt_step(p, t["r1x"], t["r1u"], t["r2"], t["r3"], t["r4"], t["sigma_s"], chol,
                    px, pu, ps, py, pz, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    code, scen = R.rkkt_status(p)
    if code != 0:
        raise RuntimeError(f"device status {code} in scenario {scen}")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # timed region 1: eager calls with per-stage HIP events on the launch stream
    R.rkkt_profile_begin(p, 16 * args.steps + 16)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    stages = R.rkkt_profile_end(p)
    eager_ms = e0.elapsed_time(e1) / args.steps
    progress(f"eager calls timed: {eager_ms:.3f} ms per pass")
    # timed region 2: the same pass captured once and replayed
    iter_args = dict(x=t["x"], u=t["u"], y=t["y"], z=t["z"], obj_weight=w, f=f, grad_x=gx,
                     grad_u=gu, g=g, h=h, sigma_x=t["sigma_x"], sigma_u=t["sigma_u"],
                     sigma_s=t["sigma_s"], delta_w=dw, khat=khat, chol=chol, info=info,
                     r1x=t["r1x"], r1u=t["r1u"], r2=t["r2"], r3=t["r3"], r4=t["r4"],
                     px=px, pu=pu, ps=ps, py=py, pz=pz)
    R.rkkt_graph_capture(p, iter_args)
    for _ in range(args.warmup):
        R.rkkt_graph_launch(p, stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        R.rkkt_graph_launch(p, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / args.steps
    progress(f"graph replays timed: {graph_ms:.3f} ms per pass")
    # the spread of single replays: the same number again with an event
    # between every two (the markers add a little to each, so these are not
    # the timed value)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for i in range(args.steps):
        R.rkkt_graph_launch(p, stream)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per_replay = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    ms = min(graph_ms, eager_ms)
    value = N / (ms * 1e-3)
    cf_ms = sum(stages[s][0] for s in ("condense_values", "refactor", "reduce", "stacked_product",
                                       "scenario_sum", "factor")) / args.steps
    dom = max((s for s in stages if stages[s][1] > 0), key=lambda s: stages[s][0])
    roof = roofline_entry(dom, stages[dom][0], stages[dom][1], d, args.config)

    out = {
        "metric": "scenario-IPM-iterations/sec (condense+factor) vs plain form; IPM iters w/ warm start",
        "value": value, "unit": "scenario-IPM-iterations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "n_scen": N, "n_x": nx, "n_u": nu, "m": m,
                   "nnz_lu": d["nnz_lu"], "col_tile": d["col_tile"], "variant": d["variant"],
                   "lds_reduce": d["lds_reduce"], "lds_group": d["lds_group"],
                   "sweep_form": d["sweep_form"], "delta_w": dw,
                   "seed": args.seed},
        "graph_ms_per_step": graph_ms, "eager_ms_per_step": eager_ms,
        "graph_replay_ms": {"median": float(np.median(per_replay)),
                            "p90": float(np.percentile(per_replay, 90)),
                            "min": float(per_replay.min()), "max": float(per_replay.max()),
                            "n": int(per_replay.size)},
        "condense_factor_value": N / (cf_ms * 1e-3),
        "stage_ms": {s: stages[s][0] / max(stages[s][1], 1) for s in stages},
        "roofline": roof,
        "roofline_pass": pass_roofline(d, ms, cf_ms),
    }

    if not args.no_probe:
        attach_probe_peaks(out, R.rkkt_probe_peaks())

    if not args.no_plain:
        # the same kernels, one scenario per handle and per launch, no batching
        handles = [R.rkkt_create(net, inst.scen.pd[:, k:k + 1].T, inst.scen.qd[:, k:k + 1].T,
                                 col_tile=args.col_tile, variant=args.variant) for k in range(N)]
        tk = [{n: t[n][k:k + 1].contiguous() for n in ("x", "y", "z", "sigma_x", "sigma_s")}
              for k in range(N)]
        su0 = zf(nu)
        kk = [zf(nu, nu) for _ in range(N)]
        f1, gx1, gu1, g1, h1 = zf(1), zf(1, nx), zf(1, nu), zf(1, nx), zf(1, m)
        kplain, cplain = zf(nu, nu), zf(nu, nu)
        eye_dw = torch.eye(nu, dtype=torch.float64, device="cuda") * dw

        for k in range(N):
            R.rkkt_evaluate(handles[k], tk[k]["x"], t["u"], tk[k]["y"], tk[k]["z"], w,
                            f1, gx1, gu1, g1, h1, stream)

        def plain():
            for k in range(N):
                R.rkkt_condense(handles[k], tk[k]["sigma_x"], su0, tk[k]["sigma_s"], dw, kk[k], stream)
            kplain.copy_(torch.diag(t["sigma_u"]) - (N - 1) * eye_dw)
            for k in range(N):
                kplain.add_(kk[k])
            cplain.copy_(kplain)
            R.rkkt_factor(handles[0], cplain, info, stream)

        plain()
        torch.cuda.synchronize()
        err = float(torch.linalg.norm(kplain - khat) / torch.linalg.norm(khat))
        n_pl = max(3, args.steps // 8)
        e0.record(stream)
        for _ in range(n_pl):
            plain()
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / n_pl
        progress(f"plain per-scenario form timed: {pms:.3f} ms per iteration")
        out["plain_form"] = {"ms_per_iteration": pms, "value": N / (pms * 1e-3),
                             "unit": "scenario-IPM-iterations/s",
                             "what": "condense launched once per scenario (N = 1 handles), "
                                     "sum of the scenario matrices, Cholesky",
                             "khat_rel_diff_vs_batched": err}
        out["speedup_condense_factor_vs_plain"] = out["condense_factor_value"] / out["plain_form"]["value"]
        del handles

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, it, dw)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
