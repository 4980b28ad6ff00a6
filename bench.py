"""Benchmark: plain per-cell burn of the 13-species / 30-reaction synthetic
network, 65,536 cells, dt = 1e-2, rtol 1e-6, atol 1e-10, FP64, one MI355X.

A step is one burn of the whole batch from the same initial state (the state
is restored from a resident copy with a device-to-device copy inside the
timed region).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 128 flop/clk x 2.4 GHz
KERNEL_SOURCES = ["paper_2312_02836_amd/csrc/burn_kernels.hip",
                  "paper_2312_02836_amd/csrc/burn_internal.h"]
TRAFFIC_FILE = "profiles/burn_plain_kernel__synth13_30__65536cells__hbm_traffic.txt"


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
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return float(kv["traffic_bytes_per_launch"])


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cells", type=int, default=65536)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--block-waves", type=int, default=0)
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

    from paper_2312_02836_amd import burn as B
    from paper_2312_02836_amd import flops, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    cfg = synth.config(2, n_cells=args.cells)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = B.Network(spec)
    Y0 = torch.as_tensor(cells.Y, device=dev).contiguous()
    T0 = torch.as_tensor(cells.T, device=dev).contiguous()
    rho = torch.as_tensor(cells.rho, device=dev).contiguous()
    Yw, Tw = Y0.clone(), T0.clone()
    st = torch.empty(args.cells, dtype=torch.int32, device=dev)
    cnt = torch.empty((8, args.cells), dtype=torch.int32, device=dev)

    from paper_2312_02836_amd import _lib
    import ctypes as C
    opts = _lib.BurnOpts(0, args.lanes, args.block_waves, 0)
    stream = torch.cuda.current_stream(dev)
    L = _lib.lib()

    def launch():
        rc = L.burn_batch_ex(net.handle, args.cells, C.c_void_p(Yw.data_ptr()),
                             C.c_void_p(rho.data_ptr()), C.c_void_p(Tw.data_ptr()), cfg.t_end,
                             cfg.rtol, cfg.atol, None, C.c_void_p(st.data_ptr()),
                             C.c_void_p(cnt.data_ptr()), C.byref(opts),
                             C.c_void_p(stream.cuda_stream))
        _lib.check(rc, "burn_batch_ex")

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

    for _ in range(args.warmup):
        Yw.copy_(Y0)
        Tw.copy_(T0)
        launch()
    torch.cuda.synchronize()
    print(f"bench: warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    k_start = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    k_end = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        Yw.copy_(Y0)
        Tw.copy_(T0)
        k_start[i].record(stream)
        launch()
        k_end[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in zip(k_start, k_end)]
    ms_per_step = 1000.0 * wall / args.steps

    status = st.cpu().numpy()
    counters = cnt.cpu().numpy()
    n_ok = int((status == 0).sum())
    value = n_ok / (ms_per_step / 1000.0)
    kernel_avg_ms = float(np.mean(kernel_ms))
    f_launch = flops.total_flops(spec, counters)
    achieved = f_launch / (kernel_avg_ms / 1000.0) / 1e12
    print(f"bench: {args.steps} steps, {ms_per_step:.3f} ms/step, kernel {kernel_avg_ms:.3f} ms "
          f"(min {min(kernel_ms):.3f}), ok {n_ok}/{args.cells}, "
          f"alg flops/launch {f_launch:.4e}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle
        onet = oracle.OracleNet(spec)
        threads = oracle.max_threads()
        n_s = 512
        rng = np.random.default_rng(1234)
        while True:
            idx = np.sort(rng.choice(cells.n_cells, min(n_s, cells.n_cells), replace=False))
            sub = cells.subset(idx)
            tc = time.perf_counter()
            oracle.burn(onet, sub, cfg.t_end, cfg.rtol, cfg.atol)
            el = time.perf_counter() - tc
            if el >= args.cpu_seconds or n_s >= cells.n_cells:
                break
            n_s = min(cells.n_cells, int(n_s * max(2.0, 1.2 * args.cpu_seconds / max(el, 1e-3))))
        cpu = {"value": len(idx) / el, "unit": "cell-burns/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(idx)} seeded random cells of the same 65,536-cell workload, "
                         f"{el:.1f} s on {threads} OpenMP threads"}

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
        "config": {"workload": "plain burn, synthetic 13-species/30-reaction network, "
                               f"{args.cells} cells, dt=1e-2, rtol 1e-6, atol 1e-10",
                   "cells": args.cells, "species": spec.n_species, "reactions": spec.n_reactions,
                   "t_end": cfg.t_end, "kernel": "burn_plain_kernel",
                   "lanes_per_cell": args.lanes or "auto"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": (measured_traffic() if (args.cells, args.lanes, args.block_waves) == (65536, 0, 0)
                                 else None),
                     "kernel_ms": kernel_avg_ms, "alg_flops_per_launch": f_launch},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    net.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
