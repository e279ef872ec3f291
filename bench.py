"""Benchmark of the MG-HLBM step on one MI355X.

A step is one structured time step of the whole hot path: lattice
interpolation nodes from the grid, lattice stream-collide, the grid's
interface donors and n finite-volume sub-steps, move + refill, wall force.
Default workload: the 2048^2 lamina case (512 x 128 grid, tau 0.55, KC 1,
beta 1000), FP64: 100 warm-up steps, the library's autotuner (which also
captures the HIP graphs the steps replay), 1000 timed steps in one call,
then 80 steps with HIP events at the stream-collide's own start and end,
80 with events at every grid sub-step launch's own start and end, and
24 steps with events around every kernel. With plain BGK this configuration
goes supersonic at the lamina tips and diverges near step 1330 (on the CPU
oracle as on the GPU), so every step stays before it.

Prints one JSON line: lattice MLUPS (whole job), a roofline entry for the
dominant kernel (the grid sub-step kernel: the largest share of the step's
GPU time; 18 s bytes per grid node and sub-step, four sub-steps per launch,
timed with HIP events on its stream; its grid is cache-resident, so the
fraction is of algorithmic bytes over the HBM peak), the same for the
lattice stream-collide (two steps per launch: the fraction of the
algorithmic bytes of both steps, and of the bytes it must move, one read and
one write of the lattice), and the CPU oracle timed on a bounded sample of
the same workload.

The "adjoint" entry times the differentiation case (1024^2 lattice, 256 x 64
grid, FP32, 4000 steps, checkpoints every 200 steps): the forward run with
checkpoints, then the discrete adjoint for the cotangent of Re Theta (window
[1, 4) periods), their time ratio, the adjoint lattice kernel against its
algorithmic bytes, and central differences of Re Theta at relative step
1e-4 in (KC, beta, tau) against the adjoint's gradient.
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES = {"f64": 8, "f32": 4, "f16dev": 2}
CALIB_COPY_BYTES = 256 << 20  # plain device copy that scales the HBM byte counters


def measured_traffic(workload, storage, kernel="k_stream_collide"):
    """HBM bytes per launch of `kernel` (a name, or a name with template
    arguments for one instance) from the committed counter summary, or None
    when there is none or the kernel source changed since."""
    from paper_2006_13631_amd.profiling import kernel_file, source_sha256
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel_file(kernel)}.{workload}.{storage}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != source_sha256() or rec.get("kernel") != kernel:
        return None
    return rec["bytes_per_launch"]


def substeps_per_launch(variant, n_sub):
    """Mean grid sub-steps per launch of a step: variants 8 and 9 advance
    one per launch, 10 two, the others up to four."""
    blk = {8: 1, 9: 1, 10: 2}.get(variant, 4)
    return n_sub / -(-n_sub // blk)


def host_cores():
    """Host threads this process may use (its CPU affinity, capped by
    OMP_NUM_THREADS when that is set)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return min(n, int(env)) if env.isdigit() and int(env) > 0 else n


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, steps):
    """The oracle as it stands on `steps` steps: single-threaded (the figure
    quoted), then with its per-node loops on every host core. Both runs must
    end in the same bits."""
    from oracle import oracle as O
    c = dict(cfg)
    c.pop("steps", None)
    c.pop("ckpt_every", None)
    runs = {}
    for threads in (1, host_cores()):
        O.set_threads(threads)
        s = O.Sim(max_steps=steps, **c)
        t0 = time.perf_counter()
        s.step(steps)
        dt = time.perf_counter() - t0
        runs[threads] = (dt, s.history(), s.lattice())
        del s
    O.set_threads(1)
    (t1, h1, f1), (tn, hn, fn) = runs[1], runs[max(runs)]
    mlups = lambda dt: c["nx"] * c["ny"] * steps / dt / 1e6
    return {"value": mlups(t1), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"first {steps} steps of the same workload, FP64, one thread ({t1:.1f} s)",
            "all_cores": {"value": mlups(tn), "cores": max(runs), "seconds": tn,
                          "same_bits": bool(np.array_equal(h1, hn) and np.array_equal(f1, fn)),
                          "nproc": os.cpu_count(), "cpu": cpu_model()}}


def oracle_timing_leg(big_steps=100, log=None):
    """The oracle timed on the host, single-threaded and with its per-node
    loops on every host core (the bits must agree): the 256x128 case and the
    128x64 copy of the differentiation case in full (the latter also with
    its complex-step derivatives along A, omega and tau, one run each), the
    2048^2 and 4096^2 workloads on their first `big_steps` steps, whose full
    runs are extrapolated from the per-step time."""
    from oracle import oracle as O
    from paper_2006_13631_amd.workloads import preset
    log = log or (lambda *a: print(*a, file=sys.stderr, flush=True))
    cores = host_cores()

    def timed(name, steps, threads, cs=None, chunk=None):
        c = preset(name)
        c.pop("steps")
        c.pop("ckpt_every", None)
        O.set_threads(threads)
        O.lib_cs().or_set_threads(threads)
        s = O.Sim(max_steps=steps, **c) if cs is None else O.SimCS(*cs, max_steps=steps, **c)
        inf = s.info()
        chunk = chunk or steps
        t, done = 0.0, 0
        while done < steps:
            n = min(chunk, steps - done)
            t0 = time.perf_counter()
            s.step(n)
            t += time.perf_counter() - t0
            done += n
            log(f"# oracle {name} threads={threads}{' complex-step' if cs else ''}: "
                f"{done}/{steps} steps, {t:.1f} s")
        node_steps = c["nx"] * c["ny"] * steps
        grid_steps = inf.n_sub * inf.nnode * steps
        row = {"seconds": t, "ms_per_step": 1e3 * t / steps, "mlups": node_steps / t / 1e6,
               "mlups_total": (node_steps + grid_steps) / t / 1e6}
        out = (s.history(), s.lattice())
        del s
        return row, out

    def same(a, b):
        return all(np.array_equal(np.asarray(x), np.asarray(y)) for x, y in zip(a, b))

    rows = {}
    plan = [("lamina_256x128", None, None), ("lamina_128x64", None, None),
            ("lamina_2048", big_steps, 10), ("lamina_4096", big_steps, 5)]
    for name, steps, chunk in plan:
        full = preset(name)["steps"]
        steps = steps or full
        r1, o1 = timed(name, steps, 1, chunk=chunk)
        rn, on = timed(name, steps, cores, chunk=chunk)
        row = {"steps": steps, "full_steps": full, "one_thread": r1, "all_cores": rn,
               "same_bits": same(o1, on)}
        del o1, on
        if steps < full:
            row["full_run_hours_extrapolated"] = {"one_thread": r1["seconds"] * full / steps / 3600,
                                                  "all_cores": rn["seconds"] * full / steps / 3600}
        rows[name] = row
    # derivatives of the differentiation copy: one complex-step run per
    # direction (A, omega, tau)
    name = "lamina_128x64"
    full = preset(name)["steps"]
    cs = {}
    for threads in (1, cores):
        tot, outs = 0.0, []
        for d in range(3):
            h = [0.0, 0.0, 0.0]
            h[d] = 1e-20
            r, o = timed(name, full, threads, cs=tuple(h))
            tot += r["seconds"]
            outs.append(o)
        cs[threads] = (tot, outs)
    rows[name]["complex_step_derivatives"] = {
        "runs": 3, "one_thread_s": cs[1][0], "all_cores_s": cs[cores][0],
        "ratio_to_forward_one_thread": cs[1][0] / rows[name]["one_thread"]["seconds"],
        "same_bits": all(same(a, b) for a, b in zip(cs[1][1], cs[cores][1]))}
    O.set_threads(1)
    O.lib_cs().or_set_threads(1)
    return {"oracle_timing": rows, "cores": cores, "nproc": os.cpu_count(), "cpu": cpu_model(),
            "build": "gcc -O2 -ffp-contract=off -fopenmp, FP64"}


def adjoint_leg(workload, storage, W_ckpt, fd_step, steps=None):
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.autograd import theta
    from paper_2006_13631_amd.workloads import preset
    cfg = preset(workload)
    full = cfg.pop("steps")
    steps = steps or full
    cfg.pop("ckpt_every", None)
    W = W_ckpt
    case = H.Case(max_steps=steps, storage=storage, ckpt_every=W, **cfg)
    info = case.info()
    sched = case.tune(trial_steps=4)
    print(f"# adjoint leg {workload} {storage} steps {steps} window {W} schedule {sched}", file=sys.stderr,
          flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    case.step(steps)
    t_fwd = time.perf_counter() - t0
    hist = torch.from_numpy(case.history()).requires_grad_(True)
    A = torch.tensor(info.A, dtype=torch.float64)
    om = torch.tensor(info.omega, dtype=torch.float64)
    th = theta(hist, A, om, cfg["b"])
    th.real.backward()
    w = hist.grad.numpy().copy()
    g = case.adjoint(w)  # first call allocates the tape
    print("# adjoint warm-up done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    g = case.adjoint(w)
    t_adj = time.perf_counter() - t0
    case.timing(True)
    case.adjoint(w)
    ms, cnt = case.timing_get(H.K_ADJ_STREAM_COLLIDE)
    ms_sub, cnt_sub = case.timing_get(H.K_ADJ_SUBSTEPS)
    case.timing(False)
    sT = BYTES[{H.FP64: "f64", H.FP32: "f32", H.FP16_DEV: "f16dev"}[storage]]
    sR = 8 if storage == H.FP64 else 4
    nodes = cfg["nx"] * cfg["ny"]
    k1_bytes = (9 * sT + 18 * sR) * nodes
    k1_avg = ms / 1000.0 / max(cnt, 1)
    # total derivative of Re Theta in (KC, beta, tau): A = KC b/(2 pi) and
    # omega = 2 pi nu beta / b^2 with nu = (tau - 1/2)/3, so tau also moves
    # omega; Theta's explicit dependence on A and omega comes from torch
    Ag = torch.tensor(info.A, dtype=torch.float64, requires_grad=True)
    omg = torch.tensor(info.omega, dtype=torch.float64, requires_grad=True)
    theta(torch.from_numpy(case.history()), Ag, omg, cfg["b"]).real.backward()
    dA, dW, dT = g[0] + Ag.grad.item(), g[1] + omg.grad.item(), g[2]
    b, tau = cfg["b"], cfg["tau"]
    adj_cfg = {"kc": dA * b / (2 * math.pi), "beta": dW * info.omega / cfg["beta"],
               "tau": dT + dW * info.omega / (tau - 0.5)}
    def central(st, rel=None):
        # central differences of Re Theta at relative step rel (fd_step)
        rel = rel or fd_step
        out = {}
        for key in (("kc", "beta", "tau") if fd_step else ()):
            vals = []
            for sgn in (1, -1):
                c2 = dict(cfg)
                c2[key] = cfg[key] * (1 + sgn * rel)
                # the sub-step count is one of the run's discrete decisions,
                # held fixed as the adjoint holds it (tau moves 1/tau_u)
                c2["n_sub"] = info.n_sub
                cc = H.Case(max_steps=steps, storage=st, **c2)
                cc.step(steps)
                vals.append(cc.theta().real)
                cc.close()
            out[key] = (vals[0] - vals[1]) / (2 * rel * cfg[key])
        return out

    def chain(grad, hist_np):
        # the adjoint's dJ/d(A, omega, tau) plus Theta's explicit dependence
        # on A and omega (torch), in (KC, beta, tau)
        Ag = torch.tensor(info.A, dtype=torch.float64, requires_grad=True)
        omg = torch.tensor(info.omega, dtype=torch.float64, requires_grad=True)
        theta(torch.from_numpy(hist_np), Ag, omg, cfg["b"]).real.backward()
        dA_, dW_, dT_ = grad[0] + Ag.grad.item(), grad[1] + omg.grad.item(), grad[2]
        return {"kc": dA_ * b / (2 * math.pi), "beta": dW_ * info.omega / cfg["beta"],
                "tau": dT_ + dW_ * info.omega / (tau - 0.5)}

    fd = central(storage)
    for key in fd:
        print(f"# fd {key}: {fd[key]:.6e} adjoint {adj_cfg[key]:.6e}", file=sys.stderr, flush=True)
    f64 = None
    if storage != H.FP64 and fd_step:
        # the same comparison in FP64, where rounding does not hide the
        # difference quotient
        c64 = H.Case(max_steps=steps, storage=H.FP64, ckpt_every=W, **cfg)
        c64.tune(trial_steps=2)
        c64.step(steps)
        h64 = torch.from_numpy(c64.history()).requires_grad_(True)
        theta(h64, torch.tensor(info.A, dtype=torch.float64), torch.tensor(info.omega, dtype=torch.float64),
              cfg["b"]).real.backward()
        adj64 = chain(c64.adjoint(h64.grad.numpy().copy()), c64.history())
        c64.close()
        fd64 = central(H.FP64)
        # a step small enough that no discrete decision of the run (node
        # status, cells, refill types) changes inside it
        fd64s = central(H.FP64, 1e-7)
        for key in fd64:
            print(f"# fp64 fd {key}: {fd64[key]:.6e} (step 1e-7: {fd64s[key]:.6e}) adjoint {adj64[key]:.6e}",
                  file=sys.stderr, flush=True)
        f64 = {"dRe_theta_dKC_beta_tau": {k: float(v) for k, v in adj64.items()},
               "fd": {k: float(v) for k, v in fd64.items()},
               "fd_rel_err": {k: float(abs(fd64[k] - adj64[k]) / abs(adj64[k])) for k in fd64},
               "fd_small_rel_step": 1e-7, "fd_small": {k: float(v) for k, v in fd64s.items()},
               "fd_small_rel_err": {k: float(abs(fd64s[k] - adj64[k]) / abs(adj64[k])) for k in fd64s}}
    return {
        "f64": f64,
        "workload": workload, "storage": {H.FP64: "f64", H.FP32: "f32", H.FP16_DEV: "f16dev"}[storage],
        "steps": steps, "ckpt_every": W, "objective": "Re Theta, window [1,4) periods",
        "forward_s": round(t_fwd, 4), "adjoint_s": round(t_adj, 4), "ratio": round(t_adj / t_fwd, 3),
        "adjoint_mlups": round(nodes * steps / t_adj / 1e6, 1),
        "grad_A_omega_tau": [float(v) for v in g],
        "dRe_theta_dKC_beta_tau": {k: float(v) for k, v in adj_cfg.items()},
        "fd_rel_step": fd_step or None, "fd": {k: float(v) for k, v in fd.items()},
        "fd_rel_err": {k: float(abs(fd[k] - adj_cfg[k]) / abs(adj_cfg[k])) for k in fd},
        "kernel": "k_adj_stream_collide", "kernel_avg_us": round(k1_avg * 1e6, 3),
        "kernel_bytes_per_launch": k1_bytes, "kernel_gbs": round(k1_bytes / k1_avg / 1e9, 1),
        "substeps_kernel": "k_adj_substeps", "substeps_launch_us": round(ms_sub * 1e3 / max(cnt_sub, 1), 3),
        "substeps_per_launch": min(4, info.n_sub),
    }


def sweep_leg(seed=0, periods=10.0, loop=True, tune_steps=8, chunk=4000, only=None, overrides=None):
    """The (KC, beta) sweep: all cases as one FP32 batch (autotuned schedule)
    against the plain FP64 loop over the same cases one by one; Theta of each
    case compared at the 1e-3 relative bar. overrides: schedule entries that
    replace the tuned ones (e.g. the persistent launch) before the run."""
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.workloads import sweep_cases
    cases, flagged = sweep_cases(seed, periods)
    if only:
        cases = [cases[i] for i in only]
        flagged = [flagged[i] for i in only]
    # a lamina faster than one lattice unit per step cannot run on the
    # lattice at all (the library rejects it): counted, not run
    speed = [c["kc"] * (c["tau"] - 0.5) / 3.0 * c["beta"] / c["b"] for c in cases]
    rejected = sum(1 for u in speed if u >= 1.0)
    keep = [i for i, u in enumerate(speed) if u < 1.0]
    cases = [cases[i] for i in keep]
    flagged = [flagged[i] for i in keep]
    n = len(cases)
    lat = sum(c["nx"] * c["ny"] * c["max_steps"] for c in cases)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch = H.Batch(cases, storage=H.FP32)
    t_create = time.perf_counter() - t0
    t0 = time.perf_counter()
    tuning = batch.tune(trial_steps=tune_steps)
    if overrides:
        sched = dict(tuning, **overrides)
        sched.pop("ms_per_step", None)
        tuning = batch.tune(schedule=sched)
    t_tune = time.perf_counter() - t0
    print(f"# sweep: {n} cases, FP32 batch, schedule {tuning}", file=sys.stderr, flush=True)
    longest = max(c["max_steps"] for c in cases)
    t0 = time.perf_counter()
    done, running, t_tail = 0, n, 0.0
    tail_n = max(1, n // 8)        # the batch's tail: at most this many cases still run
    while done < longest:
        m = min(chunk, longest - done)
        tc = time.perf_counter()
        batch.step(m)
        if running <= tail_n:
            t_tail += time.perf_counter() - tc
        done += m
        running = sum(1 for k in range(n) if batch[k].info().status == H.STATUS_RUNNING)
        print(f"# batch step {done}/{longest}, running {running}, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    t_batch = time.perf_counter() - t0

    def theta_of(member):
        try:
            return member.theta()
        except H.HlbmError as e:  # fit window holds fewer than two samples
            if e.code != H.E_ARG:
                raise
            return None
    th32 = [theta_of(batch[k]) if batch[k].info().status == H.STATUS_DONE else None for k in range(n)]
    st32 = [batch[k].info().status for k in range(n)]
    batch.close()
    out = {"metric": "parametric sweep throughput at equal force accuracy", "unit": "cases/hour",
           "higher_is_better": True, "cases": n, "rejected_speed_above_1": rejected,
           "flagged_mach": int(sum(flagged)),
           "workload": f"{n} (KC, beta) cases, seed {seed}, {periods:g} periods each, lattice 256^2..1024^2, "
                       f"grid 4b x b, b = size/8",
           "lattice_node_steps": lat,
           "batch": {"storage": "f32", "schedule": tuning, "create_s": round(t_create, 2),
                     "tune_s": round(t_tune, 2), "run_s": round(t_batch, 2),
                     "cases_per_hour": round(n / ((t_create + t_tune + t_batch) / 3600.0), 1),
                     "cases_per_hour_run_only": round(n / (t_batch / 3600.0), 1),
                     "tail_s": round(t_tail, 2), "tail_cases": tail_n,
                     "diverged": int(sum(1 for x in st32 if x == H.STATUS_UNSTABLE))}}
    out["value"] = out["batch"]["cases_per_hour"]
    if loop:
        th64, st64, t_loop = [], [], 0.0
        for k, c in enumerate(cases):
            t0 = time.perf_counter()
            g = H.Case(storage=H.FP64, **c)
            try:
                g.step(c["max_steps"])
                st64.append(H.STATUS_DONE)
            except H.HlbmError as e:
                if e.code != H.E_UNSTABLE:
                    raise
                st64.append(H.STATUS_UNSTABLE)
            th64.append(theta_of(g) if st64[-1] == H.STATUS_DONE else None)
            g.close()
            t_loop += time.perf_counter() - t0
            print(f"# fp64 loop case {k + 1}/{n} ({c['nx']}^2, {c['max_steps']} steps): {t_loop:.1f} s",
                  file=sys.stderr, flush=True)
        # equal force accuracy, case by case: a case with a Theta in FP64
        # passes when the batch gives a Theta within 1e-3 of it; a case with a
        # Theta on one side only fails
        per_case, errs = [], []
        for k, c in enumerate(cases):
            a, b = th32[k], th64[k]
            err = abs(a - b) / abs(b) if a is not None and b is not None else None
            if err is not None:
                errs.append(err)
            verdict = ("within" if err is not None and err <= 1e-3 else "outside" if err is not None
                       else "f32_only" if a is not None else "f64_only" if b is not None else "neither")
            per_case.append({"i": k, "n": c["nx"], "kc": round(c["kc"], 4), "beta": round(c["beta"], 2),
                             "tau": round(c["tau"], 4), "steps": c["max_steps"], "f32": int(st32[k]),
                             "f64": int(st64[k]), "rel_err": err, "accuracy": verdict})
        finite64 = sum(1 for b in th64 if b is not None)
        ok = sum(1 for r in per_case if r["accuracy"] == "within")
        out["loop"] = {"storage": "f64", "run_s": round(t_loop, 2),
                       "cases_per_hour": round(n / (t_loop / 3600.0), 1),
                       "diverged": int(sum(1 for x in st64 if x == H.STATUS_UNSTABLE))}
        out["speedup"] = round(out["value"] / out["loop"]["cases_per_hour"], 3)
        t_batch_all = out["batch"]["create_s"] + out["batch"]["tune_s"] + out["batch"]["run_s"]
        out["theta"] = {"finite_in_f64": finite64, "within_1e-3": ok,
                        "failures": int(sum(1 for r in per_case if r["accuracy"] in ("outside", "f32_only",
                                                                                    "f64_only"))),
                        "max_rel_err": max(errs) if errs else None,
                        "median_rel_err": float(np.median(errs)) if errs else None,
                        # the rate counting only cases whose batch Theta meets the bar
                        "batch_cases_per_hour_within": round(ok / (t_batch_all / 3600.0), 1),
                        "loop_cases_per_hour_with_theta": round(finite64 / (t_loop / 3600.0), 1)}
        out["cases_detail"] = per_case
    return out


def precision_leg(workload="lamina_4096", steps=None, chunk=1000):
    """One case at FP64, FP32 and FP16-deviation storage: lattice MLUPS of
    each, and its force history and Theta against the FP64 run (the
    hydrodynamic-function error each reduced precision costs)."""
    import math
    import numpy as np
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.workloads import preset
    cfg = preset(workload)
    cfg.pop("steps")
    cfg.pop("ckpt_every", None)
    nu = (cfg["tau"] - 0.5) / 3.0
    period = cfg["b"] ** 2 / (nu * cfg["beta"])
    steps = steps or int(math.ceil(4.0 * period)) + 1  # the fit window [T, 4T)
    runs = {}
    for st in ("f64", "f32", "f16dev"):
        case = H.Case(max_steps=steps, storage=H.STORAGE[st], **cfg)
        sched = case.tune(trial_steps=4)
        print(f"# precision {workload} {st} steps {steps} schedule {sched}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, diverged = 0, None
        while done < steps:
            n = min(chunk, steps - done)
            try:
                case.step(n)
            except H.HlbmError as e:
                if e.code != H.E_UNSTABLE:
                    raise
                diverged = case.info().step
                break
            done += n
            print(f"# {st} {done}/{steps}", file=sys.stderr, flush=True)
        dt = time.perf_counter() - t0
        hist = case.history()
        fin = np.all(np.isfinite(hist), axis=1)
        n_fin = int(np.argmin(fin)) if not fin.all() else len(hist)
        t1 = min(4.0, n_fin / period)
        th = None
        if t1 > 1.0 + 2.0 / period:
            try:
                th = case.theta(1.0, t1)
            except H.HlbmError:
                th = None
        runs[st] = {"mlups": cfg["nx"] * cfg["ny"] * (diverged or steps) / dt / 1e6, "steps_run": diverged or steps,
                    "diverged_at": diverged, "finite_steps": n_fin, "theta": th, "hist": hist[:n_fin],
                    "fit_window_periods": [1.0, t1], "schedule": sched}
        case.close()
    ref = runs["f64"]
    out = {"workload": workload, "steps": steps, "period_steps": round(period, 1)}
    n_common = min(len(r["hist"]) for r in runs.values())
    for st, r in runs.items():
        # a run that blows up does so in every precision within a few steps;
        # the force is compared over the first 90 % of the steps all kept finite
        n = int(0.9 * n_common) if n_common < steps else n_common
        scale = np.max(np.abs(ref["hist"][:n])) if n else float("nan")
        err = float(np.max(np.abs(r["hist"][:n] - ref["hist"][:n])) / scale) if n else None
        th, th64 = r["theta"], ref["theta"]
        out[st] = {"mlups": round(r["mlups"], 1), "steps_run": r["steps_run"], "diverged_at": r["diverged_at"],
                   "theta": None if th is None else [th.real, th.imag],
                   "fit_window_periods": [round(x, 3) for x in r["fit_window_periods"]],
                   "force_rel_err_vs_f64": err, "force_compared_steps": n,
                   "theta_rel_err_vs_f64": None if (th is None or th64 is None) else abs(th - th64) / abs(th64),
                   "schedule": {k: r["schedule"][k] for k in ("lattice_threads", "lattice_rows", "substep_variant", "order")}}
    return out


def paper_theta(eps, beta):
    """The paper's own MG-HLBM Theta for one of its (epsilon, beta) cases
    (Figs. aggregate_re and aggregate_im, 4 decimals; tests/golden), or
    None for a pair it did not run."""
    path = os.path.join(ROOT, "tests", "golden", "paper_mg_hlbm_theta.txt")
    for line in open(path):
        f = line.split("#")[0].split()
        if len(f) == 4 and abs(float(f[0]) - eps) < 1e-12 and int(f[1]) == int(round(beta)):
            return complex(float(f[2]), -float(f[3]))
    return None


def study_leg(b=64, storage="f64", tune_steps=8, chunk=2000):
    """The paper's (epsilon, beta) study (35 pairs under Eq.(betalimit), 5L x 5L
    domain, the paper's outer boundaries) as one batch; Theta of each case
    beside the semianalytical values the paper compares with (context: a
    different discretisation and resolution, not a parity bar)."""
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.theory import theta_semianalytical
    from paper_2006_13631_amd.workloads import paper_study_cases
    cases = paper_study_cases(b=b)
    cfgs = [{k: v for k, v in c.items() if k not in ("eps", "beta_p")} for c in cases]
    t0 = time.perf_counter()
    batch = H.Batch(cfgs, storage=H.STORAGE[storage])
    sched = batch.tune(trial_steps=tune_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    longest = max(c["max_steps"] for c in cfgs)
    done = 0
    while done < longest:
        n = min(chunk, longest - done)
        batch.step(n)
        done += n
        print(f"# study {done}/{longest} steps", file=sys.stderr, flush=True)
    batch[0].info()
    t2 = time.perf_counter()
    rows = []
    devs_re, devs_im = [], []
    pdev_re, pdev_im = [], []
    for i, c in enumerate(cases):
        inf = batch[i].info()
        th = batch[i].theta() if inf.status == H.STATUS_DONE else None
        ref = theta_semianalytical(c["beta_p"], c["eps"])
        row = {"eps": c["eps"], "beta": c["beta_p"], "steps": c["max_steps"], "status": int(inf.status),
               "theta": None if th is None else [round(th.real, 5), round(th.imag, 5)],
               "semianalytical": [round(ref.real, 5), round(ref.imag, 5)]}
        pap = paper_theta(c["eps"], c["beta_p"])
        if pap is not None:
            row["paper_mg_hlbm"] = [pap.real, pap.imag]
        if th is not None:
            row["dev_re"] = round((th.real - ref.real) / ref.real, 4)
            row["dev_im"] = round((th.imag - ref.imag) / ref.imag, 4)
            devs_re.append(abs(row["dev_re"]))
            devs_im.append(abs(row["dev_im"]))
            if pap is not None:
                row["dev_paper_re"] = round((th.real - pap.real) / pap.real, 4)
                row["dev_paper_im"] = round((th.imag - pap.imag) / pap.imag, 4)
                pdev_re.append(abs(row["dev_paper_re"]))
                pdev_im.append(abs(row["dev_paper_im"]))
        rows.append(row)
    import statistics
    return {"metric": "the paper's (epsilon, beta) study: Theta per case, cases/hour", "unit": "cases/hour",
            "storage": storage, "cases": len(cases), "lattice": f"{5 * b}^2 (5L x 5L), L = {b}",
            "grid": f"{4 * b} x {b}", "bc": "paper (no-slip x walls, outflow y ends)",
            "tau": [round(min(c["tau"] for c in cases), 4), round(max(c["tau"] for c in cases), 4)], "schedule": sched, "setup_s": round(t1 - t0, 2), "run_s": round(t2 - t1, 2),
            "value": round(len(cases) / ((t2 - t0) / 3600.0), 1),
            "median_abs_dev_re": statistics.median(devs_re) if devs_re else None,
            "median_abs_dev_im": statistics.median(devs_im) if devs_im else None,
            "median_abs_dev_paper_re": statistics.median(pdev_re) if pdev_re else None,
            "median_abs_dev_paper_im": statistics.median(pdev_im) if pdev_im else None, "per_case": rows}


def levels_leg(b=800, nlevels=4, storage="f64", steps=40, warmup=4, uniform=True):
    """The paper's structured refinement: 4 levels over a 5L x 5L domain, the
    lamina (L = 800 at the finest resolution, the paper's value) on the
    finest. Times level-0 steps (2^(levels-1) finest steps each) replayed as
    HIP graphs, and the same lamina, grid and finest resolution on one
    uniform lattice over the whole domain, per finest step."""
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.workloads import paper_levels
    d = paper_levels(b=b, nlevels=nlevels)
    per = 2 ** (nlevels - 1)
    fine = dict(d["fine"])
    m = H.MultiLevel(d["nx0"], d["ny0"], d["boxes"], bc0=d["bc0"], storage=H.STORAGE[storage],
                     max_steps=(steps + warmup) * per, **fine)
    sched = m.tune(trial_steps=4)
    inf = m.info()
    print(f"# levels {m.shapes} taus {m.taus} n_sub {inf.n_sub} schedule {sched}", file=sys.stderr, flush=True)
    m.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nodes = [nx * ny * 2 ** l for l, (nx, ny) in enumerate(m.shapes)]
    grid_sub = inf.nnode * inf.n_sub * per
    out = {"workload": f"paper_levels_{b}", "storage": storage, "levels": [
        {"nx": nx, "ny": ny, "tau": round(t, 6), "steps_per_level0_step": 2 ** l, "box": list(bx) if l < len(d["boxes"]) else None}
        for l, ((nx, ny), t, bx) in enumerate(zip(m.shapes, m.taus, d["boxes"] + [None]))],
        "grid": [fine["nux"], fine["nuy"]], "n_sub": inf.n_sub, "level0_steps": steps,
        "ms_per_level0_step": round(dt / steps * 1e3, 4), "ms_per_finest_step": round(dt / steps / per * 1e3, 4),
        "mlups_levels": round(sum(nodes) * steps / dt / 1e6, 1),
        "mlups_total": round((sum(nodes) + grid_sub) * steps / dt / 1e6, 1),
        "schedule": {k: sched[k] for k in ("lattice_threads", "lattice_rows", "substep_variant", "order")}}
    m.close()
    if uniform:
        n = 5 * b + 1
        c = H.Case(nx=n, ny=n, bc=H.BC_PAPER, storage=H.STORAGE[storage], max_steps=(steps + warmup) * per, **fine)
        c.tune(trial_steps=4)
        c.step(warmup * per)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(steps * per)
        torch.cuda.synchronize()
        du = time.perf_counter() - t0
        c.close()
        out["uniform"] = {"nx": n, "ny": n, "ms_per_step": round(du / (steps * per) * 1e3, 4),
                          "mlups": round(n * n * steps * per / du / 1e6, 1)}
        out["speedup_vs_uniform"] = round(du / dt, 3)
    return out


def levels_theta_leg(b=256, nlevels=4, eps=0.1, beta=20.0, tau=0.8, storage="f64", periods=4.2, chunk=2048,
                     uniform=True, n_sub=0):
    """Theta of the lamina on the finest of the paper's refinement levels
    against one uniform lattice at the finest resolution over the same
    5L x 5L domain (same grid, tau, boundaries), and the time each takes;
    the semianalytical value of the paper's Eqs. (hydro_gamma),(hydro_delta)
    and, for one of its cases, the paper's own MG-HLBM value beside them as
    context."""
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.theory import theta_semianalytical
    from paper_2006_13631_amd.workloads import paper_levels
    d = paper_levels(b=b, nlevels=nlevels, eps=eps, beta=beta, tau=tau, margin=8)
    if n_sub:
        d["fine"]["n_sub"] = n_sub  # grid sub-steps per step (0: the smallest stable count)
    per = 2 ** (nlevels - 1)
    nu = (tau - 0.5) / 3.0
    period = b * b / (nu * beta)  # finest steps
    n0 = int(math.ceil(periods * period / per))
    runs = {}
    for kind in ("levels", "uniform") if uniform else ("levels",):
        if kind == "levels":
            c = H.MultiLevel(d["nx0"], d["ny0"], d["boxes"], bc0=d["bc0"], storage=H.STORAGE[storage],
                             max_steps=n0 * per, **d["fine"])
            total, unit = n0, per
        else:
            n = 5 * b + 1
            c = H.Case(nx=n, ny=n, bc=H.BC_PAPER, storage=H.STORAGE[storage], max_steps=n0 * per, **d["fine"])
            total, unit = n0 * per, 1
        c.tune(trial_steps=4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < total:
            k = min(chunk, total - done)
            c.step(k)
            done += k
            print(f"# levels theta {kind} {done}/{total}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        th = c.theta(1.0, 4.0)
        runs[kind] = {"theta": [th.real, th.imag], "s": round(dt, 3),
                      "ms_per_finest_step": round(dt / (total * unit) * 1e3, 4)}
        runs[kind]["n_sub"] = int(c.info().n_sub)
        if kind == "levels":
            runs[kind]["levels"] = [list(sh) for sh in c.shapes]
        else:
            runs[kind]["lattice"] = [5 * b + 1, 5 * b + 1]
        c.close()
    tl = complex(*runs["levels"]["theta"])
    ts = theta_semianalytical(beta, eps)
    out = {"workload": f"paper_levels_{b}_theta", "storage": storage, "nlevels": nlevels, "eps": eps,
           "beta": beta, "tau_finest": tau, "grid": [4 * b, b],
           "finest_steps": n0 * per, "period_steps": round(period, 1), **runs,
           "theta_semianalytical": [ts.real, ts.imag]}
    if uniform:
        tu = complex(*runs["uniform"]["theta"])
        out["theta_rel_diff_levels_vs_uniform"] = abs(tl - tu) / abs(tu)
        out["speedup_vs_uniform"] = round(runs["uniform"]["s"] / runs["levels"]["s"], 3)
    pap = paper_theta(eps, beta)
    if pap is not None:
        out["theta_paper_mg_hlbm"] = [pap.real, pap.imag]
        out["theta_rel_diff_levels_vs_paper"] = abs(tl - pap) / abs(pap)
    return out


def coupled_leg(workload="lamina_2048", storage="f64", periods=2.5, mass_ratio=1.0, chunk=1000):
    """The workload's lattice and grid with the lamina elastically mounted
    instead of driven: released from y0 = b/16, spring set so that the
    undamped period in vacuum is the workload's forcing period, mass
    mass_ratio times (pi/4) rho b^2. Lattice MLUPS of the coupled steps
    (the same kernels plus the motion update) beside the prescribed-motion
    run of the main line, and the free decay: mean half period and
    amplitude ratio per half period over the first swings."""
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.workloads import preset
    cfg = preset(workload)
    cfg.pop("steps")
    cfg.pop("ckpt_every", None)
    b = cfg["b"]
    nu = (cfg["tau"] - 0.5) / 3.0
    omega = 2 * math.pi * nu * cfg["beta"] / (b * b)
    period = 2 * math.pi / omega
    steps = int(periods * period)
    M = mass_ratio * math.pi / 4 * b * b
    K = M * omega * omega
    A = cfg["kc"] * b / (2 * math.pi)
    case = H.Case(storage=H.STORAGE[storage], max_steps=steps, **cfg)
    case.set_motion(M, K, 0.0, y0=b / 16, v0=0.0, y_max=max(abs(A), b / 8))
    sched = case.tune(trial_steps=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        case.step(n)
        done += n
        print(f"# coupled {done}/{steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    y = case.motion_history()[:, 0]
    case.close()
    zc = np.where(np.diff(np.sign(y)) != 0)[0]
    halves = np.diff(zc[:6]) if len(zc) > 2 else np.array([])
    peaks = [float(np.abs(y[zc[i]:zc[i + 1]]).max()) for i in range(min(len(zc) - 1, 5))]
    ratios = [peaks[i + 1] / peaks[i] for i in range(len(peaks) - 1)]
    return {"workload": workload + "_coupled", "storage": storage, "steps": steps,
            "mass": M, "stiffness": K, "y0": b / 16, "vacuum_period_steps": round(period, 1),
            "mlups": round(cfg["nx"] * cfg["ny"] * steps / dt / 1e6, 1), "ms_per_step": round(1e3 * dt / steps, 4),
            "half_periods": [int(h) for h in halves], "peak_ratios": [round(r, 4) for r in ratios],
            "schedule": {k: sched[k] for k in ("lattice_threads", "lattice_rows", "substep_variant", "order")}}


def graded_leg(workload="lamina_1024", storage="f64"):
    """The workload's lamina on its uniform grid (spacing 1) and on a graded
    grid over the same extent (spacing 1 over the lamina, growing to 2 away
    from it: about half the nodes): time per step and Theta over [T, 4T)."""
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.workloads import graded_nodes, preset
    cfg = preset(workload)
    steps = cfg.pop("steps")
    cfg.pop("ckpt_every", None)
    half_x = cfg["nux"] // 2 * cfg["h_u"]
    half_y = 0.5 * (cfg["nuy"] - 1) * cfg["h_u"]
    nx_, ny_ = 5, 4
    while graded_nodes(nx_, 1.0, 1.04, 2.0, fine=0.6 * cfg["b"])[-1] < half_x:
        nx_ += 2
    while graded_nodes(ny_, 1.0, 1.06, 2.0, fine=4.0)[-1] < half_y:
        ny_ += 2
    gx = graded_nodes(nx_, 1.0, 1.04, 2.0, fine=0.6 * cfg["b"])
    gy = graded_nodes(ny_, 1.0, 1.06, 2.0, fine=4.0)
    out = {"workload": workload, "storage": storage, "steps": steps}
    thetas = {}
    for kind in ("uniform", "graded"):
        kw = dict(cfg, storage=H.STORAGE[storage], max_steps=steps)
        if kind == "graded":
            kw.update(nux=nx_, nuy=ny_, x_nodes=gx, y_nodes=gy)
        c = H.Case(**kw)
        c.tune(trial_steps=4)
        c.step(8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(steps - 8)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        th = c.theta(1.0, 4.0)
        thetas[kind] = th
        out[kind] = {"grid": [kw["nux"], kw["nuy"]], "grid_nodes": c.info().nnode,
                     "ms_per_step": round(1e3 * dt / (steps - 8), 4),
                     "mlups": round(cfg["nx"] * cfg["ny"] * (steps - 8) / dt / 1e6, 1),
                     "theta": [th.real, th.imag]}
        print(f"# graded leg {kind}: {out[kind]}", file=sys.stderr, flush=True)
        c.close()
    out["theta_rel_diff"] = abs(thetas["graded"] - thetas["uniform"]) / abs(thetas["uniform"])
    out["speedup"] = round(out["uniform"]["ms_per_step"] / out["graded"]["ms_per_step"], 3)
    return out


def mesh_leg(workload="lamina_2048", storage="f64", steps=200, warmup=20, timing_steps=40, h_wall=1.0, seed=1,
             bend=0.0):
    """The workload's lamina on an unstructured Delaunay grid of the same
    extent (spacing h_wall on the lamina growing to 1, seeded) against its
    split-quad grid: time per step, the CSR sub-step kernel's mean launch
    time (its own events, one sub-step per launch) against its algorithmic
    bytes (the stencil's neighbours read and the node written, 9 values
    each), and the lattice MLUPS. The mesh grid is L2-resident, so the
    achieved rate is not an HBM fraction. bend != 0: also the unstructured
    grid with its lamina bending at amplitude `bend` (the grid's weights,
    triangles and wall edges rebuilt every step)."""
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.meshes import lamina_triangulation
    from paper_2006_13631_amd.workloads import preset
    cfg = preset(workload)
    cfg.pop("steps")
    cfg.pop("ckpt_every", None)
    W = (cfg["nux"] - 1) * cfg["h_u"]
    Hh = (cfg["nuy"] - 1) * cfg["h_u"]
    t0 = time.perf_counter()
    mesh = lamina_triangulation(W, Hh, b=cfg["b"], T=cfg["thickness"], h_wall=h_wall, h_far=1.0, seed=seed)
    t_mesh = time.perf_counter() - t0
    tri = mesh[2]
    edges = np.unique(np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]), axis=1), axis=0)
    entries = len(mesh[0]) + 2 * len(edges)  # stencil entries: the node and its neighbours
    s_b = BYTES[storage]
    out = {"workload": workload, "storage": storage, "steps": steps,
           "mesh": {"W": W, "H": Hh, "h_wall": h_wall, "h_far": 1.0, "seed": seed, "nodes": len(mesh[0]),
                    "triangles": int(len(tri)), "mean_stencil": round(entries / len(mesh[0]), 3),
                    "generate_s": round(t_mesh, 2)}}
    total = warmup + steps + timing_steps
    for kind in ("split_quad", "unstructured") + (("bending",) if bend else ()):
        kw = dict(cfg, storage=H.STORAGE[storage], max_steps=total)
        if kind != "split_quad":
            kw["mesh"] = mesh
        c = H.Case(**kw)
        if kind == "bending":
            c.set_deformation(bend, 0.0)
        c.step(warmup)
        sched = c.tune(trial_steps=4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        c.timing(3)
        c.step(timing_steps)
        ms_g, n_g = c.timing_get(H.K_SUBSTEP_LAUNCH)
        c.timing(0)
        inf = c.info()
        avg_g = ms_g / 1000.0 / max(n_g, 1)
        rec = {"grid_nodes": inf.nnode, "n_sub": inf.n_sub, "ms_per_step": round(1e3 * dt / steps, 4),
               "mlups": round(cfg["nx"] * cfg["ny"] * steps / dt / 1e6, 1),
               "substep_launch_us": round(avg_g * 1e6, 3), "launches_timed": n_g,
               "schedule": {k: sched[k] for k in ("lattice_threads", "lattice_rows", "substep_variant", "order")}}
        if kind != "split_quad":
            byts = (entries + inf.nnode) * 9 * s_b  # stencil reads + one write per node
            rec.update({"substeps_per_launch": 1, "bytes_per_launch": byts,
                        "achieved_gbs": round(byts / avg_g / 1e9, 1), "kernel": f"k_mesh_substep<{storage}>"})
        else:
            per = substeps_per_launch(sched["substep_variant"], inf.n_sub)
            byts = int(round(18 * s_b * inf.nnode * per))
            rec.update({"substeps_per_launch": per, "bytes_per_launch": byts,
                        "achieved_gbs": round(byts / avg_g / 1e9, 1),
                        "kernel": f"k_grid_substeps<{storage}, {sched['substep_variant']}>"})
        out[kind] = rec
        print(f"# mesh leg {kind}: {rec}", file=sys.stderr, flush=True)
        c.close()
    return out


def storage_leg(workload, storage, steps, warmup, timing_steps):
    """The same workload at another storage precision: lattice MLUPS over
    graph-replayed steps, the stream-collide's mean duration (its own events)
    against its algorithmic bytes, and Theta over the steps run."""
    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.workloads import preset
    cfg = preset(workload)
    case = H.case_from_preset(cfg, storage=storage, max_steps=warmup + steps + 2 * timing_steps)
    case.step(warmup)
    sched = case.tune(trial_steps=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    case.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    case.timing(2)
    case.step(timing_steps)
    ms, n = case.timing_get(H.K_STREAM_COLLIDE)
    case.timing(3)
    case.step(timing_steps)
    ms_g, n_g = case.timing_get(H.K_SUBSTEP_LAUNCH)
    case.timing(0)
    info = case.info()
    nodes = cfg["nx"] * cfg["ny"]
    avg = ms / 1000.0 / max(n, 1)
    gbs = 18 * BYTES[storage] * nodes / avg / 1e9
    per_launch = substeps_per_launch(sched["substep_variant"], info.n_sub)
    avg_g = ms_g / 1000.0 / max(n_g, 1)
    grid_gbs = 18 * {"f64": 8}.get(storage, 4) * info.nnode * per_launch / avg_g / 1e9
    th = None
    try:
        th = case.theta()
    except H.HlbmError:
        pass
    two = bool(case.info().two_step)
    return {"storage": storage, "value": round(nodes * steps / dt / 1e6, 2), "unit": "MLUPS",
            "ms_per_step": round(1000.0 * dt / steps, 4),
            "stream_collide_kernel": "k_stream_collide2" if two else "k_stream_collide",
            "stream_collide_steps_per_launch": 2 if two else 1, "stream_collide_us": round(avg * 1e6, 3),
            "stream_collide_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "substep_launch_us": round(avg_g * 1e6, 3), "substep_gbs": round(grid_gbs, 1),
            "substep_frac": round(grid_gbs / HBM_PEAK_GBS, 4),
            "theta": None if th is None else [th.real, th.imag],
            "schedule": {k: sched[k] for k in ("lattice_threads", "lattice_rows", "substep_variant", "order")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="lamina_2048")
    ap.add_argument("--storage", default="f64", choices=list(BYTES))
    ap.add_argument("--timing-steps", type=int, default=80,
                    help="event-timed steps of the stream-collide, then as many of the grid sub-steps")
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--adjoint-workload", default="lamina_1024")
    ap.add_argument("--adjoint-storage", default="f32", choices=list(BYTES))
    ap.add_argument("--adjoint-window", type=int, default=200)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=None)
    ap.add_argument("--no-fd", action="store_true")
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32 line of the main workload")
    ap.add_argument("--sweep", action="store_true",
                    help="run only the parametric sweep (FP32 batch vs FP64 per-case loop) and print its line")
    ap.add_argument("--sweep-periods", type=float, default=10.0)
    ap.add_argument("--sweep-no-loop", action="store_true")
    ap.add_argument("--sweep-schedule", default=None,
                    help="JSON object of schedule entries replacing the tuned ones (e.g. persistent)")
    ap.add_argument("--precision", action="store_true",
                    help="run only the storage-precision comparison (FP64 / FP32 / FP16-deviation) and print its line")
    ap.add_argument("--precision-workload", default="lamina_4096,lamina_4096_stable")
    ap.add_argument("--precision-steps", type=int, default=None)
    ap.add_argument("--study", action="store_true",
                    help="run only the paper's (epsilon, beta) study as one batch and print its line")
    ap.add_argument("--study-b", type=int, default=64)
    ap.add_argument("--study-storage", default="f64", choices=list(BYTES))
    ap.add_argument("--levels", action="store_true",
                    help="run only the paper's 4-level refinement (L = 800 on the finest level) against a "
                         "uniform finest lattice and print its line")
    ap.add_argument("--levels-storage", default="f64", choices=list(BYTES))
    ap.add_argument("--levels-steps", type=int, default=40)
    ap.add_argument("--levels-no-uniform", action="store_true")
    ap.add_argument("--graded", action="store_true",
                    help="run only the differentiation case on its uniform grid and on a graded grid of the same "
                         "extent and print their line")
    ap.add_argument("--mesh", action="store_true",
                    help="run only the main workload on an unstructured Delaunay grid against its split-quad grid "
                         "and print their line")
    ap.add_argument("--mesh-steps", type=int, default=200)
    ap.add_argument("--mesh-bend", type=float, default=0.0,
                    help="with --mesh: also run the unstructured grid with the lamina bending at this amplitude")
    ap.add_argument("--coupled", action="store_true",
                    help="run only the main workload with the lamina elastically mounted (two-way coupled) and "
                         "print its line")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="run only the oracle's host timing (one thread and all host cores) on the four "
                         "workloads and print its line")
    ap.add_argument("--oracle-steps", type=int, default=100)
    ap.add_argument("--levels-theta", action="store_true",
                    help="run only Theta on 4 refinement levels (L = 256 at the finest) against a uniform "
                         "finest lattice over the same domain and print its line")
    ap.add_argument("--lt-b", type=int, default=256, help="--levels-theta: L at the finest level")
    ap.add_argument("--lt-eps", type=float, default=0.1)
    ap.add_argument("--lt-beta", type=float, default=20.0)
    ap.add_argument("--lt-tau", type=float, default=0.8, help="--levels-theta: tau at the finest level")
    ap.add_argument("--lt-periods", type=float, default=4.2)
    ap.add_argument("--lt-no-uniform", action="store_true")
    ap.add_argument("--lt-n-sub", type=int, default=0, help="--levels-theta: grid sub-steps per step (0: auto)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)
    if args.oracle_timing:
        print(json.dumps(oracle_timing_leg(args.oracle_steps)), flush=True)
        return

    import torch
    from paper_2006_13631_amd import hlbm as H
    from paper_2006_13631_amd.workloads import preset

    if args.sweep:
        torch.cuda.set_device(0)
        over = json.loads(args.sweep_schedule) if args.sweep_schedule else None
        print(json.dumps(sweep_leg(periods=args.sweep_periods, loop=not args.sweep_no_loop, overrides=over)),
              flush=True)
        return
    if args.graded:
        torch.cuda.set_device(0)
        print(json.dumps(graded_leg()), flush=True)
        return
    if args.mesh:
        torch.cuda.set_device(0)
        print(json.dumps(mesh_leg(args.workload, args.storage, steps=args.mesh_steps, bend=args.mesh_bend)), flush=True)
        return
    if args.coupled:
        torch.cuda.set_device(0)
        print(json.dumps(coupled_leg(args.workload, args.storage)), flush=True)
        return
    if args.levels_theta:
        torch.cuda.set_device(0)
        print(json.dumps(levels_theta_leg(b=args.lt_b, eps=args.lt_eps, beta=args.lt_beta, tau=args.lt_tau,
                                          storage=args.levels_storage, periods=args.lt_periods,
                                          uniform=not args.lt_no_uniform, n_sub=args.lt_n_sub)), flush=True)
        return
    if args.levels:
        torch.cuda.set_device(0)
        print(json.dumps(levels_leg(storage=args.levels_storage, steps=args.levels_steps,
                                    uniform=not args.levels_no_uniform)), flush=True)
        return
    if args.study:
        torch.cuda.set_device(0)
        print(json.dumps(study_leg(args.study_b, args.study_storage)), flush=True)
        return
    if args.precision:
        torch.cuda.set_device(0)
        for wl in args.precision_workload.split(","):
            print(json.dumps(precision_leg(wl, args.precision_steps)), flush=True)
        return

    cfg = preset(args.workload)
    steps = args.steps if args.steps is not None else min(cfg["steps"], 1000)
    W = args.warmup
    detail_steps = 24
    total = W + steps + 2 * args.timing_steps + detail_steps
    torch.cuda.set_device(0)
    # a plain copy of known size, so counter runs of this command can scale
    # the HBM byte counters (not part of any timed region)
    src = torch.empty(CALIB_COPY_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    case = H.case_from_preset(cfg, storage=args.storage, max_steps=total)
    info = case.info()
    print(f"# workload {args.workload} storage {args.storage} n_sub {info.n_sub} "
          f"grid nodes {info.nnode} warmup {W} steps {steps}", file=sys.stderr, flush=True)

    case.step(W)
    # launch shapes picked by the library's autotuner (state untouched); it
    # also captures the HIP graphs of the steps that follow
    sched = case.tune(trial_steps=4)
    print(f"# schedule {sched}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    case.step(steps)  # one call: whole graphs replayed, one wait at the end
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"# {steps} timed steps in {dt:.4f} s", file=sys.stderr, flush=True)
    nx, ny = cfg["nx"], cfg["ny"]
    mlups = nx * ny * steps / dt / 1e6

    # the stream-collide's own start and end events on its stream, nothing
    # else recorded in these steps (on the two-step path: the launch that
    # advances the lattice outside the band by two steps, reading it once and
    # writing it once)
    two = bool(case.info().two_step)
    case.timing(2)
    case.step(args.timing_steps)
    ms_k1, n_k1 = case.timing_get(H.K_STREAM_COLLIDE)
    # the first grid sub-step launch of each step (of each pair on the
    # two-step path), its own start and end events, nothing else recorded
    case.timing(3)
    case.step(args.timing_steps)
    ms_g, n_g = case.timing_get(H.K_SUBSTEP_LAUNCH)
    # then every kernel (events between all kernels; informational)
    case.timing(1)
    case.step(detail_steps)
    kern = {}
    for name, kid in (("stream_collide", H.K_STREAM_COLLIDE), ("lattice_from_grid", H.K_LATTICE_FROM_GRID),
                      ("grid_substeps", H.K_GRID_SUBSTEPS), ("refill", H.K_REFILL), ("force", H.K_FORCE),
                      ("step", H.K_STEP)):
        ms, cnt = case.timing_get(kid)
        kern[name] = round(1000.0 * ms / max(cnt, 1), 3)
    case.timing(0)
    s_b = BYTES[args.storage]
    avg_s = ms_k1 / 1000.0 / max(n_k1, 1)
    lat_bytes = 18 * s_b * nx * ny  # one read and one write of the lattice
    spl = 2 if two else 1
    lat_kernel = "k_stream_collide2" if two else "k_stream_collide"
    # the grid sub-step kernel: 18 s bytes per node and sub-step, the
    # launch's sub-steps (4, or n when fewer)
    per_launch = substeps_per_launch(sched["substep_variant"], info.n_sub)
    grid_kernel = f"k_grid_substeps<{ {'f64': 'double'}.get(args.storage, 'float') }, {sched['substep_variant']}>"
    avg_g = ms_g / 1000.0 / max(n_g, 1)
    grid_bytes = int(round(18 * s_b * info.nnode * per_launch))
    grid_achieved = grid_bytes / avg_g / 1e9
    th = None
    try:
        th = case.theta()
    except H.HlbmError:
        pass

    out = {
        "metric": "lattice MLUPS (whole MG-HLBM step) + HBM roofline fraction of the dominant kernel",
        "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": W,
        "ms_per_step": round(1000.0 * dt / steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": args.workload, "nx": nx, "ny": ny, "nux": cfg["nux"], "nuy": cfg["nuy"],
                   "b": cfg["b"], "tau": cfg["tau"], "kc": cfg["kc"], "beta": cfg["beta"],
                   "n_sub": info.n_sub, "storage": args.storage,
                   "schedule": {k: sched[k] for k in ("lattice_threads", "lattice_rows", "substep_variant", "order")}},
        # the dominant kernel: the grid sub-steps (n launches' worth per step
        # against the lattice's one); its grid stays in L2 and the memory-side
        # cache, so this is algorithmic bytes over the HBM peak
        "roofline": {"bound": "hbm", "achieved": round(grid_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(grid_achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.workload, args.storage, grid_kernel),
                     "kernel": grid_kernel, "substeps_per_launch": per_launch,
                     "launches_per_step": round(info.n_sub / per_launch), "avg_us": round(avg_g * 1e6, 3),
                     "bytes_per_launch": grid_bytes, "resident": "L2 + memory-side cache"},
        # the lattice stream-collide: `frac` prices a launch at the
        # algorithmic bytes of the steps it advances (18 s per node update);
        # `frac_moved` at the bytes it must move, one read and one write
        "lattice": {"kernel": lat_kernel, "steps_per_launch": spl, "avg_us": round(avg_s * 1e6, 3),
                    "us_per_step": round(avg_s * 1e6 / spl, 3),
                    "bytes_per_launch": spl * lat_bytes,
                    "achieved": round(spl * lat_bytes / avg_s / 1e9, 1),
                    "frac": round(spl * lat_bytes / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                    "moved_bytes_per_launch": lat_bytes,
                    "frac_moved": round(lat_bytes / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(args.workload, args.storage, lat_kernel)},
        "kernel_avg_us": kern,
        "mlups_total": round((nx * ny + info.n_sub * info.nnode) * steps / dt / 1e6, 2),
        "theta": None if th is None else [th.real, th.imag],
    }
    case.close()
    if args.storage == "f64" and not args.no_f32:
        # the sweep-scale configuration is quoted at FP64 and FP32
        out["f32"] = storage_leg(args.workload, "f32", steps, W, args.timing_steps)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(args.adjoint_workload, H.STORAGE[args.adjoint_storage], args.adjoint_window,
                                     0.0 if args.no_fd else 1e-4, args.adjoint_steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
