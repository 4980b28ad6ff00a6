"""Benchmark of the per-cell reaction burn on one MI355X (FP64, rtol 1e-6).

Workloads (--workload):
  synth13  (default) burn of the synthetic 13-species / 30-reaction
           network, 65,536 cells, dt = 1e-2, one persistent launch (a lane
           group that finishes a cell takes the next from a device work
           queue), with the plain launch (static map of cells to lane groups)
           timed beside it;
  mixed4   four networks (13/30, 21/60, 35/100, 50/150), 65,536 cells each,
           in ONE persistent launch with a device work queue; the plain
           kernel (one launch per network) is timed beside it;
  synth50  the 50-species / 150-reaction network, 1,048,576 cells, one
           persistent launch, with the plain launch timed beside it;
  adjoint21  sensitivities of the 21-species / 60-reaction network, 65,536
           cells: recording burn, replay with exact correctors and reverse
           sweep (16-step checkpoints) per step, one random cotangent of all
           end abundances and E per cell; metric: adjoint grads/s.

A step is one burn of the whole batch from the same initial state (the state
is restored from a resident copy with device-to-device copies inside the
timed region, outside the kernel events).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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
KERNEL_SOURCES = ["paper_2312_02836_amd/csrc/burn_body.h",
                  "paper_2312_02836_amd/csrc/bn_math.h",
                  "paper_2312_02836_amd/csrc/burn_plain.h",
                  "paper_2312_02836_amd/csrc/burn_multi.hip",
                  "paper_2312_02836_amd/csrc/burn_internal.h"]
TRAFFIC_FILE = "profiles/burn_multi_kernel__synth13_30__65536cells__hbm_traffic.txt"

WORKLOADS = {
    "synth13": dict(config=2, cells=65536, mode="persistent",
                    text="burn of one synthetic 13-species/30-reaction network, {cells} cells, "
                         "dt=1e-2, rtol 1e-6, atol 1e-10"),
    "mixed4": dict(config=4, cells=65536, mode="persistent",
                   text="mixed persistent burn, synthetic 13/30 + 21/60 + 35/100 + 50/150 "
                        "species/reaction networks, {cells} cells each in one launch, dt=1e-2, "
                        "rtol 1e-6, atol 1e-10"),
    "adjoint21": dict(config=5, cells=65536, mode="adjoint",
                      text="adjoint sensitivities, synthetic 21-species/60-reaction network, "
                           "{cells} cells, gradient of all end abundances and E with respect to "
                           "60 log-rate multipliers, dt=1e-2, rtol 1e-6, atol 1e-10, checkpoint "
                           "every 16 steps"),
    "synth50": dict(config=3, cells=1048576, mode="persistent",
                    text="persistent burn, synthetic 50-species/150-reaction network, {cells} "
                         "cells, T log-uniform [0.8, 6], dt=1e-2, rtol 1e-6, atol 1e-10"),
}


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the burn kernel from the committed FETCH_SIZE /
    WRITE_SIZE passes, or None when the kernel sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
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
    return float(kv["traffic_bytes_per_launch"])


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="synth13")
    ap.add_argument("--cells", type=int, default=0, help="cells per network (0 = workload's)")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--block-waves", type=int, default=0)
    ap.add_argument("--mode", choices=["plain", "persistent"], default=None,
                    help="override the workload's launch mode")
    ap.add_argument("--no-compare", action="store_true",
                    help="time only the workload's schedule (not the other one beside it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size before the warmup "
                         "(calibrates FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the burn needs no communication; "
              f"--gpus {args.gpus} is not supported)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2312_02836_amd import _lib
    from paper_2312_02836_amd import burn as B
    from paper_2312_02836_amd import flops, synth

    wl = dict(WORKLOADS[args.workload])
    if args.mode:
        wl["mode"] = args.mode
    n_cells = args.cells or wl["cells"]
    if wl["mode"] == "adjoint":
        return bench_adjoint(args, wl, n_cells)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    cfg = synth.config(wl["config"], n_cells=n_cells)
    L = _lib.lib()
    stream = torch.cuda.current_stream(dev)

    # resident inputs and working copies, per network
    batches = []
    for spec, cells in zip(cfg.networks, cfg.cells):
        net = B.Network(spec)
        if args.lanes:
            net.set_launch(*_shape_for(spec.n, args.lanes), args.block_waves)
        b = dict(spec=spec, cells=cells, net=net,
                 Y0=torch.as_tensor(cells.Y, device=dev).contiguous(),
                 T0=torch.as_tensor(cells.T, device=dev).contiguous(),
                 rho=torch.as_tensor(cells.rho, device=dev).contiguous())
        b["Yw"], b["Tw"] = b["Y0"].clone(), b["T0"].clone()
        b["st"] = torch.empty(n_cells, dtype=torch.int32, device=dev)
        b["cnt"] = torch.empty((8, n_cells), dtype=torch.int32, device=dev)
        batches.append(b)
    opts = _lib.BurnOpts(0, 0, args.block_waves, 0)

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

    multi = None
    if wl["mode"] == "persistent" or not args.no_compare:
        multi = B.MultiBurn([(b["net"], b["Yw"], b["rho"], b["Tw"]) for b in batches], cfg.t_end,
                            cfg.rtol, cfg.atol, block_waves=args.block_waves)
        for b, o in zip(batches, multi.outputs):  # MultiBurn owns its status/counter tensors
            b["st_m"], b["cnt_m"] = o[2], o[3]

    def step_persistent():
        multi.run()

    def step_plain():
        for b in batches:
            launch_plain(b)

    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"bench: copy probe {nb} bytes read + {nb} bytes written", file=sys.stderr,
              flush=True)
        del src, dst

    def timed(step, label):
        for _ in range(args.warmup):
            restore()
            step()
        torch.cuda.synchronize()
        print(f"bench: {label}: warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
        ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            restore()
            ev0[i].record(stream)
            step()
            ev1[i].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
        print(f"bench: {label}: {args.steps} steps, {1000 * wall / args.steps:.3f} ms/step, "
              f"kernel {np.mean(kms):.3f} ms (min {min(kms):.3f})", file=sys.stderr, flush=True)
        return 1000.0 * wall / args.steps, float(np.mean(kms))

    other = None  # (schedule, ms/step, kernel ms) of the schedule timed beside
    if wl["mode"] == "plain":
        if not args.no_compare:
            other = ("persistent",) + timed(step_persistent, "persistent (one launch)")
        ms_per_step, kernel_ms = timed(step_plain, "plain")
        outs = [(b["st"], b["cnt"]) for b in batches]
        kernel_name = "burn_plain_kernel"
    else:
        if not args.no_compare:
            other = ("plain",) + timed(step_plain, "plain (one launch per network)")
        ms_per_step, kernel_ms = timed(step_persistent, "persistent (one launch)")
        outs = [(b["st_m"], b["cnt_m"]) for b in batches]
        kernel_name = "burn_multi_kernel"

    n_ok, f_launch = 0, 0.0
    for b, (st, cnt) in zip(batches, outs):
        s = st.cpu().numpy()
        n_ok += int((s == 0).sum())
        f_launch += flops.total_flops(b["spec"], cnt.cpu().numpy())
    n_total = n_cells * len(batches)
    value = n_ok / (ms_per_step / 1000.0)
    achieved = f_launch / (kernel_ms / 1000.0) / 1e12
    print(f"bench: ok {n_ok}/{n_total}, alg flops/launch {f_launch:.4e}", file=sys.stderr,
          flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batches, cfg, args.cpu_seconds)

    traffic = None
    if (args.workload == "synth13" and wl["mode"] == "persistent"
            and (n_cells, args.lanes, args.block_waves) == (65536, 0, 0)):
        traffic = measured_traffic()
    config = {"workload": wl["text"].format(cells=n_cells), "cells_per_network": n_cells,
              "networks": [f"{b['spec'].n_species}/{b['spec'].n_reactions}" for b in batches],
              "t_end": cfg.t_end, "kernel": kernel_name,
              "launch": [list(b["net"].get_launch()) for b in batches]}
    config[f"{'plain' if wl['mode'] == 'plain' else 'persistent'}_kernel_ms"] = kernel_ms
    if other is not None:
        config[f"{other[0]}_kernel_ms"] = other[2]
        # the persistent launch against one plain launch per network
        pers = kernel_ms if wl["mode"] == "persistent" else other[2]
        plain = kernel_ms if wl["mode"] == "plain" else other[2]
        config["persistent_vs_plain"] = plain / pers
    out = {
        "metric": "cell-burns/s (FP64, rtol 1e-6)",
        "value": value,
        "unit": "cell-burns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": config,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": traffic, "kernel_ms": kernel_ms,
                     "alg_flops_per_launch": f_launch},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    for b in batches:
        b["net"].close()
    return 0


def bench_adjoint(args, wl, n_cells) -> int:
    import numpy as np
    import torch

    from paper_2312_02836_amd import burn as B
    from paper_2312_02836_amd import flops, synth

    torch.cuda.set_device(0)
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

    def step():
        run.forward()
        return run.backward(gY, gE)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"bench: adjoint: warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
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
    ms_per_step = 1000.0 * wall / args.steps
    st = run.status.cpu().numpy()
    n_ok = int((st == 0).sum())
    f_launch = float(flops.adjoint_cell_flops(spec, run.counters.cpu().numpy(),
                                              run.replay_iters.cpu().numpy())[st == 0].sum())
    achieved = f_launch / (kernel_ms / 1000.0) / 1e12
    print(f"bench: adjoint: {args.steps} steps, {ms_per_step:.3f} ms/step (forward {fwd_ms:.3f}, "
          f"backward {bwd_ms:.3f}), ok {n_ok}/{n_cells}, alg flops/step {f_launch:.4e}",
          file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle
        onet = oracle.OracleNet(spec)
        threads = oracle.max_threads()
        k = 64
        rng = np.random.default_rng(1234)
        while True:
            idx = np.sort(rng.choice(n_cells, min(k, n_cells), replace=False))
            tc = time.perf_counter()
            oracle.sens(onet, cells.subset(idx), cfg.t_end, cfg.rtol, cfg.atol)
            el = time.perf_counter() - tc
            if el >= args.cpu_seconds or k >= n_cells:
                break
            k = min(n_cells, int(k * max(2.0, 1.2 * args.cpu_seconds / max(el, 1e-3))))
        cpu = {"value": len(idx) / el, "unit": "grads/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(idx)} seeded random cells of the same workload, forward "
                         f"sensitivities (all {spec.n_reactions} multipliers), {el:.1f} s on "
                         f"{threads} OpenMP threads"}
    out = {
        "metric": "adjoint grads/s (cell VJPs, FP64, rtol 1e-6)",
        "value": n_ok / (ms_per_step / 1000.0),
        "unit": "grads/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["text"].format(cells=n_cells), "cells": n_cells,
                   "networks": [f"{spec.n_species}/{spec.n_reactions}"], "t_end": cfg.t_end,
                   "kernel": "adjoint_kernel (+ burn_record_kernel)", "forward_ms": fwd_ms,
                   "backward_ms": bwd_ms, "max_steps": 1024},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel_ms": kernel_ms, "alg_flops_per_launch": f_launch},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    del grad
    net.close()
    return 0


def _shape_for(n: int, lanes: int):
    """Smallest padded shape with the given lanes per cell."""
    for L_, S_ in ((4, 1), (4, 2), (4, 4), (8, 4), (16, 2), (32, 1), (16, 4), (32, 2), (64, 1)):
        if L_ == lanes and L_ * S_ >= n:
            return L_, S_
    raise SystemExit(f"no shape with {lanes} lanes per cell for a system of size {n}")


def cpu_baseline(batches, cfg, seconds: float):
    """The oracle on the host cores, on a seeded sample of the same cells
    (the same fraction of every network), scaled to cell-burns/s."""
    import numpy as np
    from oracle import oracle
    threads = oracle.max_threads()
    onets = [oracle.OracleNet(b["spec"]) for b in batches]
    C_ = batches[0]["cells"].n_cells
    frac = min(1.0, 512.0 / C_)
    rng = np.random.default_rng(1234)
    while True:
        k = max(1, int(round(frac * C_)))
        idx = np.sort(rng.choice(C_, k, replace=False))
        tc = time.perf_counter()
        for b, on in zip(batches, onets):
            oracle.burn(on, b["cells"].subset(idx), cfg.t_end, cfg.rtol, cfg.atol)
        el = time.perf_counter() - tc
        if el >= seconds or frac >= 1.0:
            break
        frac = min(1.0, frac * max(2.0, 1.2 * seconds / max(el, 1e-3)))
    n = k * len(batches)
    return {"value": n / el, "unit": "cell-burns/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} seeded random cells of each of the {len(batches)} network(s) of the "
                      f"same workload ({n} cells), {el:.1f} s on {threads} OpenMP threads"}


if __name__ == "__main__":
    sys.exit(main())
