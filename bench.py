"""Benchmark of the per-cell reaction burn on one MI355X (FP64, rtol 1e-6).

The headline (the one JSON line's top-level fields) is the burn of the
synthetic 13-species / 30-reaction network, 65,536 cells, dt = 1e-2, in one
persistent launch (a lane group that finishes a cell takes the next from a
device work queue, stiffest cells first), with the plain launch (static map of
cells to lane groups) timed beside it.  The same line carries, under
"sub_results", the other workloads, each timed here the same way:

  robertson3  Robertson-like 3-species / 4-reaction network, 256 cells,
              t_end 1e3 (plain launch: 256 cells fill a fraction of the GPU,
              and a persistent grid sized to the GPU only adds its set-up;
              the persistent launch is timed beside it);
  mixed4      four networks (13/30, 21/60, 35/100, 50/150), 65,536 cells
              each, in one persistent launch; plain launches beside it;
  synth50_1M  the 50/150 network, 1,048,576 cells whose step counts vary
              tenfold, persistent launch captured into a HIP graph and
              replayed; plain launch beside it;
  adjoint21   sensitivities of the 21/60 network, 65,536 cells: recording
              burn, replay with exact correctors, reverse sweep with 16-step
              checkpoints, one random cotangent of all end abundances and E
              per cell (adjoint grads/s).

A step is one burn of the whole batch from the same initial state (restored
from a resident copy with device-to-device copies inside the timed region,
outside the kernel events).  Inputs are resident in HBM before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-sub]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2312_02836_amd/csrc/burn_gen_body.h",
                  "paper_2312_02836_amd/csrc/burn_gen_args.h",
                  "paper_2312_02836_amd/csrc/burn_codegen.cpp",
                  "paper_2312_02836_amd/csrc/burn_body.h",
                  "paper_2312_02836_amd/csrc/bn_math.h",
                  "paper_2312_02836_amd/csrc/burn_plain.h",
                  "paper_2312_02836_amd/csrc/burn_multi.hip",
                  "paper_2312_02836_amd/csrc/burn_internal.h"]
TRAFFIC_FILE = "profiles/bn_gen_burn__synth13_30__65536cells__hbm_traffic.txt"
SQ_FILE = "profiles/bn_gen_burn__synth13_30__65536cells__sq_counters.txt"

WORKLOADS = {
    "synth13": dict(config=2, cells=65536, mode="persistent", body="generated",
                    text="burn of one synthetic 13-species/30-reaction network, {cells} cells, "
                         "dt=1e-2, rtol 1e-6, atol 1e-10"),
    "robertson3": dict(config=1, cells=256, mode="plain",
                       text="plain burn of the Robertson-like 3-species/4-reaction network, "
                            "{cells} cells, t_end=1e3, rtol 1e-6, atol 1e-10"),
    "mixed4": dict(config=4, cells=65536, mode="persistent", body="generated",
                   text="mixed persistent burn, synthetic 13/30 + 21/60 + 35/100 + 50/150 "
                        "species/reaction networks, {cells} cells each in one launch, dt=1e-2, "
                        "rtol 1e-6, atol 1e-10"),
    "synth50": dict(config=3, cells=1048576, mode="persistent", graph=True,
                    text="persistent burn, synthetic 50-species/150-reaction network, {cells} "
                         "cells, T log-uniform [0.8, 6], t_end=3e-4 (step counts p95/p5 ~ 10), "
                         "rtol 1e-6, atol 1e-10, HIP graph replay"),
    "adjoint21": dict(config=5, cells=65536, mode="adjoint",
                      text="adjoint sensitivities, synthetic 21-species/60-reaction network, "
                           "{cells} cells, gradient of all end abundances and E with respect to "
                           "60 log-rate multipliers, dt=1e-2, rtol 1e-6, atol 1e-10, checkpoint "
                           "every 16 steps"),
}
# sub-results of the default run: (name, workload, timed steps, warmup steps)
SUBS = [("robertson3", "robertson3", 5, 1), ("mixed4", "mixed4", 3, 1),
        ("synth50_1M", "synth50", 3, 1), ("adjoint21", "adjoint21", 3, 1)]


def log(msg: str) -> None:
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_values(rel: str):
    """The `key = value` lines of a committed profile summary, or None when
    the kernel sources changed since it was taken (its recorded hash)."""
    path = os.path.join(ROOT, rel)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.split("#")[0].strip()
    if kv.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return kv


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# burn workloads
# ---------------------------------------------------------------------------

def run_burn(wl_name: str, steps: int, warmup: int, args, compare: bool, cpu_seconds: float,
             one_thread_seconds: float = 0.0) -> dict:
    import numpy as np
    import torch

    from paper_2312_02836_amd import _lib
    from paper_2312_02836_amd import burn as B
    from paper_2312_02836_amd import flops, synth

    wl = dict(WORKLOADS[wl_name])
    if args.mode and wl_name == args.workload:
        wl["mode"] = args.mode
    n_cells = (args.cells if wl_name == args.workload and args.cells else 0) or wl["cells"]
    dev = torch.device("cuda", 0)
    cfg = synth.config(wl["config"], n_cells=n_cells)
    L = _lib.lib()
    stream = torch.cuda.current_stream(dev)
    log(f"{wl_name}: {len(cfg.networks)} network(s), {n_cells} cells each")

    batches = []
    for spec, cells in zip(cfg.networks, cfg.cells):
        net = B.Network(spec)
        if args.lanes and wl_name == args.workload:
            net.set_launch(*_shape_for(spec.n, args.lanes), args.block_waves)
        b = dict(spec=spec, cells=cells, net=net,
                 Y0=torch.as_tensor(cells.Y, device=dev).contiguous(),
                 T0=torch.as_tensor(cells.T, device=dev).contiguous(),
                 rho=torch.as_tensor(cells.rho, device=dev).contiguous())
        b["Yw"], b["Tw"] = b["Y0"].clone(), b["T0"].clone()
        b["st"] = torch.empty(n_cells, dtype=torch.int32, device=dev)
        b["cnt"] = torch.empty((8, n_cells), dtype=torch.int32, device=dev)
        batches.append(b)
    # the generated kernel where the workload asks for it and the system
    # size allows (compiled, or taken from the cache, outside the timed region)
    body = args.body if (args.body and wl_name == args.workload) else wl.get("body", "table")
    gen = []
    if body == "generated" and wl["mode"] != "adjoint":
        for b in batches:
            if b["spec"].n <= 16 and b["spec"].screen is None:
                t0 = time.perf_counter()
                lanes = b["net"].generate()
                gen.append({"network": f"{b['spec'].n_species}/{b['spec'].n_reactions}",
                            "lanes_per_cell": lanes,
                            "seconds": round(time.perf_counter() - t0, 2)})
                log(f"{wl_name}: generated kernel for {gen[-1]['network']}, {lanes} lanes per "
                    f"cell ({gen[-1]['seconds']} s)")
    opts = _lib.BurnOpts(0, 0, args.block_waves, 0)
    # the persistent kernel's launch choice per network: from the tuning
    # cache, or tuned on the first 65,536 cells (outside the timed region)
    tune = []
    if not args.no_tune and not (args.lanes or args.block_waves):
        for b in batches:
            k = min(65536, n_cells)
            t0 = time.perf_counter()
            e = B.tune_cached(b["net"], b["Y0"][:, :k].contiguous(), b["rho"][:k].contiguous(),
                              b["T0"][:k].contiguous(), cfg.t_end, cfg.rtol, cfg.atol)
            tune.append({"network": f"{b['spec'].n_species}/{b['spec'].n_reactions}",
                         "choice": e["persistent"], "cache_hit": e["hit"],
                         "sample_cells": e["sample_cells"],
                         "seconds": round(time.perf_counter() - t0, 2)})
            log(f"{wl_name}: persistent choice {e['persistent']} "
                f"({'cache' if e['hit'] else 'tuned'})")
            if wl["mode"] == "plain":
                # the plain launch shape too (timed on the same sample)
                t0 = time.perf_counter()
                B.autotune(b["net"], b["Y0"][:, :k].contiguous(), b["rho"][:k].contiguous(),
                           b["T0"][:k].contiguous(), cfg.t_end, cfg.rtol, cfg.atol)
                tune[-1]["plain_choice"] = list(b["net"].get_launch())
                tune[-1]["plain_seconds"] = round(time.perf_counter() - t0, 2)
                log(f"{wl_name}: plain choice {tune[-1]['plain_choice']}")

    def restore():
        for b in batches:
            b["Yw"].copy_(b["Y0"])
            b["Tw"].copy_(b["T0"])

    def launch_plain(b):
        rc = L.burn_batch_ex(b["net"].handle, n_cells, C.c_void_p(b["Yw"].data_ptr()),
                             C.c_void_p(b["rho"].data_ptr()), C.c_void_p(b["Tw"].data_ptr()),
                             cfg.t_end, cfg.rtol, cfg.atol, None, C.c_void_p(b["st"].data_ptr()),
                             C.c_void_p(b["cnt"].data_ptr()), C.byref(opts),
                             C.c_void_p(stream.cuda_stream))
        _lib.check(rc, "burn_batch_ex")

    multi = B.MultiBurn([(b["net"], b["Yw"], b["rho"], b["Tw"]) for b in batches], cfg.t_end,
                        cfg.rtol, cfg.atol, block_waves=args.block_waves)
    for b, o in zip(batches, multi.outputs):  # MultiBurn owns its status/counter tensors
        b["st_m"], b["cnt_m"] = o[2], o[3]
    use_graph = bool(wl.get("graph")) and wl["mode"] == "persistent"
    if use_graph:
        restore()
        multi.capture()

    def step_persistent():
        if use_graph:
            multi.replay()
        else:
            multi.run()

    def step_plain():
        for b in batches:
            launch_plain(b)

    def timed(step, label, n_steps, n_warm):
        for _ in range(n_warm):
            restore()
            step()
        torch.cuda.synchronize()
        log(f"{wl_name} {label}: warmup done ({n_warm} steps)")
        ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(n_steps)]
        ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(n_steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n_steps):
            restore()
            ev0[i].record(stream)
            step()
            ev1[i].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
        log(f"{wl_name} {label}: {n_steps} steps, {1000 * wall / n_steps:.3f} ms/step, kernel "
            f"{np.mean(kms):.3f} ms (min {min(kms):.3f})")
        return 1000.0 * wall / n_steps, float(np.mean(kms))

    def set_body(name):
        for b in batches:
            if b["net"].body[1]:
                b["net"].set_body(name)

    other, table_pers = None, None
    if wl["mode"] == "plain":
        if compare:
            other = ("persistent",) + timed(step_persistent, "persistent", max(1, steps // 2), 1)
        ms_per_step, kernel_ms = timed(step_plain, "plain", steps, warmup)
        outs = [(b["st"], b["cnt"]) for b in batches]
        kernel_name = "burn_plain_kernel"
    else:
        if compare:
            # the table-driven kernels beside the generated one: plain
            # launches, and the persistent launch when a network has a
            # generated kernel
            set_body("table")
            other = ("plain",) + timed(step_plain, "plain table kernels (one launch per network)",
                                       max(1, min(steps, 5) // 2 if use_graph else steps),
                                       1 if use_graph else warmup)
            if gen:
                table_pers = timed(step_persistent, "persistent, table kernels only",
                                   max(1, steps // 2), 1)
            set_body("generated")
        ms_per_step, kernel_ms = timed(step_persistent,
                                       "persistent (graph replay)" if use_graph else
                                       "persistent (one launch" +
                                       (", generated kernels)" if gen else ")"), steps, warmup)
        outs = [(b["st_m"], b["cnt_m"]) for b in batches]
        kernel_name = "bn_gen_burn" if gen and len(gen) == len(batches) else (
            "bn_gen_burn + burn_multi_kernel" if gen else "burn_multi_kernel")

    n_ok, f_path, f_ext, step_stats = 0, 0.0, 0.0, []
    for b, (st, cnt) in zip(batches, outs):
        s, c = st.cpu().numpy(), cnt.cpu().numpy()
        n_ok += int((s == 0).sum())
        f_path += flops.path_total_flops(b["spec"], c)
        f_ext += flops.total_flops(b["spec"], c)
        step_stats.append((float(c[0].mean()), float(np.percentile(c[0], 5)),
                         float(np.percentile(c[0], 95))))
    n_total = n_cells * len(batches)
    value = n_ok / (ms_per_step / 1000.0)
    achieved = f_path / (kernel_ms / 1000.0) / 1e12
    alg_bytes = sum(n_cells * (8 * (2 * b["spec"].n_species + 3) + 4) for b in batches)
    log(f"{wl_name}: ok {n_ok}/{n_total}, path-model flops/launch {f_path:.4e}")

    roof = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "kernel_ms": kernel_ms,
            "alg_flops_per_launch": f_path,
            "extended_model": {"alg_flops_per_launch": f_ext,
                               "achieved": f_ext / (kernel_ms / 1000.0) / 1e12,
                               "frac": f_ext / (kernel_ms / 1000.0) / 1e12 / FP64_PEAK_TFLOPS},
            "alg_hbm_gbs": alg_bytes / (kernel_ms / 1000.0) / 1e9,
            "alg_hbm_frac": alg_bytes / (kernel_ms / 1000.0) / 1e9 / HBM_PEAK_GBS}
    config = {"workload": wl["text"].format(cells=n_cells), "cells_per_network": n_cells,
              "networks": [f"{b['spec'].n_species}/{b['spec'].n_reactions}" for b in batches],
              "t_end": cfg.t_end, "kernel": kernel_name, "graph_replay": use_graph,
              "launch": [list(b["net"].get_launch()) for b in batches],
              "persistent_launch": [list(b["net"].get_persistent_launch()) for b in batches],
              "persistent_tuning": tune, "generated": gen,
              "steps_mean_p5_p95": step_stats}
    config[f"{'plain' if wl['mode'] == 'plain' else 'persistent'}_kernel_ms"] = kernel_ms
    if other is not None:
        config[f"{other[0]}_kernel_ms"] = other[2]
        pers = kernel_ms if wl["mode"] == "persistent" else other[2]
        plain = kernel_ms if wl["mode"] == "plain" else other[2]
        config["persistent_vs_plain"] = plain / pers
    if table_pers is not None:
        config["table_persistent_kernel_ms"] = table_pers[1]
        config["generated_vs_table_persistent"] = table_pers[1] / kernel_ms
    cpu = None
    if cpu_seconds > 0:
        cpu = cpu_baseline(batches, cfg, cpu_seconds, one_thread_seconds)
    res = {"metric": "cell-burns/s (FP64, rtol 1e-6)", "value": value, "unit": "cell-burns/s",
           "steps": steps, "warmup": warmup, "ms_per_step": ms_per_step, "dtype": "f64",
           "config": config, "roofline": roof, "cpu_baseline": cpu}
    del multi
    for b in batches:
        b["net"].close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


# OpenMP threads of the host (read once: a one-thread run sets the default
# for the rest of the process)
_ALL_THREADS = None


def all_threads() -> int:
    global _ALL_THREADS
    if _ALL_THREADS is None:
        from oracle import oracle
        _ALL_THREADS = oracle.max_threads()
    return _ALL_THREADS


def cpu_baseline(batches, cfg, seconds: float, one_thread_seconds: float = 0.0):
    """The oracle on the host cores, on a seeded sample of the same cells
    (the same cells of every network), scaled to cell-burns/s: on all the
    OpenMP threads, and (when one_thread_seconds > 0) on one thread."""
    import numpy as np
    from oracle import oracle
    onets = [oracle.OracleNet(b["spec"]) for b in batches]
    C_ = batches[0]["cells"].n_cells

    def timed_sample(budget, threads):
        """(cells per network, seconds per pass over them, passes timed)."""
        frac = min(1.0, 64.0 / C_)
        rng = np.random.default_rng(1234)

        def one_pass(idx):
            tc = time.perf_counter()
            for b, on in zip(batches, onets):
                oracle.burn(on, b["cells"].subset(idx), cfg.t_end, cfg.rtol, cfg.atol,
                            n_threads=threads)
            return time.perf_counter() - tc

        while True:
            k = max(1, int(round(frac * C_)))
            idx = np.sort(rng.choice(C_, k, replace=False))
            el = one_pass(idx)
            if el >= budget:
                return k, el, 1
            if frac >= 1.0:
                # the whole workload takes less than the budget: the first
                # pass warms up, then passes are repeated until they fill it
                times = []
                while sum(times) < budget and len(times) < 1000:
                    times.append(one_pass(idx))
                return k, sum(times) / len(times), len(times)
            frac = min(1.0, frac * max(2.0, 1.2 * budget / max(el, 1e-3)))

    threads = all_threads()
    k, el, passes = timed_sample(seconds, threads)
    n = k * len(batches)
    rep = f", mean of {passes} passes after a warm-up pass" if passes > 1 else ""
    out = {"value": n / el, "unit": "cell-burns/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{k} seeded random cells of each of the {len(batches)} network(s) of the "
                     f"same workload ({n} cells), {el:.3g} s per pass on {threads} OpenMP "
                     f"threads{rep}"}
    if one_thread_seconds > 0:
        k1, el1, p1 = timed_sample(one_thread_seconds, 1)
        out["value_1thread"] = k1 * len(batches) / el1
        out["sample_1thread"] = (f"{k1 * len(batches)} cells, {el1:.3g} s per pass on 1 thread"
                                 + (f", mean of {p1} passes after a warm-up pass" if p1 > 1 else ""))
    log(f"cpu baseline: {out['value']:.1f} cell-burns/s on {threads} threads"
        + (f", {out['value_1thread']:.1f} on 1" if "value_1thread" in out else ""))
    return out


# ---------------------------------------------------------------------------
# adjoint workload
# ---------------------------------------------------------------------------

def run_adjoint(steps: int, warmup: int, n_cells: int, cpu_seconds: float) -> dict:
    import numpy as np
    import torch

    from paper_2312_02836_amd import burn as B
    from paper_2312_02836_amd import flops, synth

    wl = WORKLOADS["adjoint21"]
    dev = torch.device("cuda", 0)
    cfg = synth.config(wl["config"], n_cells=n_cells)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = B.Network(spec)
    run = B.AdjointRun(net, cells.Y, cells.rho, cells.T, cfg.t_end, cfg.rtol, cfg.atol,
                       max_steps=1024, device=dev)
    rng = np.random.default_rng(5)
    gY = torch.as_tensor(rng.normal(size=(spec.n_species, n_cells)), device=dev)
    gE = torch.as_tensor(rng.normal(size=n_cells), device=dev)
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        run.forward()
        run.backward(gY, gE)
    torch.cuda.synchronize()
    # the workspace's state pool sized from the recorded steps (outside the
    # timed region)
    if warmup:
        run.fit_pool()
    log(f"adjoint21: warmup done ({warmup} steps), state pool {run.pool_steps} steps")
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev0[i].record(stream)
        run.forward()
        ev1[i].record(stream)
        grad = run.backward(gY, gE)
        ev2[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)]))
    bwd_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(ev1, ev2)]))
    kernel_ms = fwd_ms + bwd_ms
    ms_per_step = 1000.0 * wall / steps
    st = run.status.cpu().numpy()
    n_ok = int((st == 0).sum())
    # cells whose corrected states the pool held were not recomputed
    recomp = run.pool_steps < run.recorded_steps()
    f_launch = float(flops.adjoint_cell_flops(spec, run.counters.cpu().numpy(),
                                              run.replay_iters.cpu().numpy(),
                                              recomputed=recomp)[st == 0].sum())
    achieved = f_launch / (kernel_ms / 1000.0) / 1e12
    log(f"adjoint21: {steps} steps, {ms_per_step:.3f} ms/step (forward {fwd_ms:.3f}, backward "
        f"{bwd_ms:.3f}), ok {n_ok}/{n_cells}")
    cpu = None
    if cpu_seconds > 0:
        from oracle import oracle
        onet = oracle.OracleNet(spec)
        threads = all_threads()
        k = 64
        rng = np.random.default_rng(1234)
        while True:
            idx = np.sort(rng.choice(n_cells, min(k, n_cells), replace=False))
            tc = time.perf_counter()
            oracle.sens(onet, cells.subset(idx), cfg.t_end, cfg.rtol, cfg.atol,
                        n_threads=threads)
            el = time.perf_counter() - tc
            if el >= cpu_seconds or k >= n_cells:
                break
            k = min(n_cells, int(k * max(2.0, 1.2 * cpu_seconds / max(el, 1e-3))))
        cpu = {"value": len(idx) / el, "unit": "grads/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"{len(idx)} seeded random cells of the same workload, forward "
                         f"sensitivities (all {spec.n_reactions} multipliers), {el:.1f} s on "
                         f"{threads} OpenMP threads"}
    del grad
    net.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return {"metric": "adjoint grads/s (cell VJPs, FP64, rtol 1e-6)",
            "value": n_ok / (ms_per_step / 1000.0), "unit": "grads/s", "steps": steps,
            "warmup": warmup, "ms_per_step": ms_per_step, "dtype": "f64",
            "config": {"workload": wl["text"].format(cells=n_cells), "cells": n_cells,
                       "networks": [f"{spec.n_species}/{spec.n_reactions}"], "t_end": cfg.t_end,
                       "kernel": "adjoint_kernel (+ burn_record_kernel)", "forward_ms": fwd_ms,
                       "backward_ms": bwd_ms, "max_steps": 1024,
                       "workspace_bytes": int(run.ws.numel()),
                       "workspace_min_bytes": int(run.ws_min),
                       "state_pool_steps": int(run.pool_steps)},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                         "traffic": None, "kernel_ms": kernel_ms,
                         "alg_flops_per_launch": f_launch,
                         "flop_model": "recording burn + replay (iterations x (RHS + "
                                       "solve), factorizations x (Jacobian + LU)) + per step "
                                       "the reverse terms (+ a second replay for cells "
                                       "outside the state pool)"},
            "cpu_baseline": cpu}


def _shape_for(n: int, lanes: int):
    """Smallest padded shape with the given lanes per cell."""
    for L_, S_ in ((4, 1), (4, 2), (4, 4), (8, 4), (16, 2), (32, 1), (16, 4), (32, 2), (64, 1)):
        if L_ == lanes and L_ * S_ >= n:
            return L_, S_
    raise SystemExit(f"no shape with {lanes} lanes per cell for a system of size {n}")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="synth13")
    ap.add_argument("--cells", type=int, default=0, help="cells per network (0 = workload's)")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--block-waves", type=int, default=0)
    ap.add_argument("--body", choices=["generated", "table"], default=None,
                    help="kernels of the headline workload (default: the workload's)")
    ap.add_argument("--mode", choices=["plain", "persistent"], default=None,
                    help="override the workload's launch mode")
    ap.add_argument("--no-compare", action="store_true",
                    help="time only the workload's schedule (not the other one beside it)")
    ap.add_argument("--no-sub", action="store_true", help="headline workload only")
    ap.add_argument("--no-tune", action="store_true",
                    help="persistent launches with the derived (untuned) choice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-seconds-1thread", type=float, default=8.0)
    ap.add_argument("--sub-cpu-seconds", type=float, default=4.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size before the warmup "
                         "(calibrates FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the burn needs no communication between "
              f"GPUs; --gpus {args.gpus} is not supported)", file=sys.stderr)
        return 2

    import torch
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe {nb} bytes read + {nb} bytes written")
        del src, dst

    if not args.no_cpu_baseline:
        all_threads()
    cpu_s = 0.0 if args.no_cpu_baseline else args.cpu_seconds
    cpu1_s = 0.0 if args.no_cpu_baseline else args.cpu_seconds_1thread
    sub_cpu = 0.0 if args.no_cpu_baseline else args.sub_cpu_seconds
    if WORKLOADS[args.workload]["mode"] == "adjoint" and args.mode is None:
        head = run_adjoint(args.steps, args.warmup,
                           args.cells or WORKLOADS["adjoint21"]["cells"], cpu_s)
    else:
        head = run_burn(args.workload, args.steps, args.warmup, args, not args.no_compare,
                        cpu_s, cpu1_s)

    if args.workload == "synth13" and head["roofline"]["kernel_ms"] > 0:
        default_launch = (not args.cells and not args.lanes and not args.block_waves
                          and not args.mode and args.body in (None, "generated"))
        tr = profile_values(TRAFFIC_FILE) if default_launch else None
        if tr is not None:
            head["roofline"]["traffic"] = float(tr["traffic_bytes_per_launch"])
        sq = profile_values(SQ_FILE) if default_launch else None
        if sq is not None:
            cf = float(sq["fp64_flops_per_dispatch"])
            kms = float(sq["kernel_ms"])
            head["roofline"]["counter_fp64_tflops"] = cf / (kms / 1000.0) / 1e12
            head["roofline"]["counter_fp64_frac"] = cf / (kms / 1000.0) / 1e12 / FP64_PEAK_TFLOPS
            head["roofline"]["simt_efficiency"] = head["roofline"]["alg_flops_per_launch"] / cf

    sub = {}
    if not args.no_sub and args.workload == "synth13":
        for name, wl_name, st, wu in SUBS:
            if WORKLOADS[wl_name]["mode"] == "adjoint":
                sub[name] = run_adjoint(st, wu, WORKLOADS[wl_name]["cells"], sub_cpu)
            else:
                sub[name] = run_burn(wl_name, st, wu, args, True, sub_cpu)

    out = {
        "metric": head["metric"],
        "value": head["value"],
        "unit": head["unit"],
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": head["cpu_baseline"],
    }
    if sub:
        out["sub_results"] = sub
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
