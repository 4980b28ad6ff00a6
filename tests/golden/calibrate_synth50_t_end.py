"""Calibration of the burn time of the 50-species / 150-reaction workload.

That workload stands for cells of uneven stiffness whose step counts vary
about tenfold.  Its burn time t_end is therefore chosen so that the ratio of
the 95th to the 5th percentile of the oracle's accepted-step counts, on a
seeded 4,096-cell sample of its cells, is about 10 (rtol 1e-6, atol 1e-10).
This script calls only the oracle and the seeded input generator; it writes
synth50_t_end.txt next to itself.  synth.config(3) holds the chosen value and
tests/test_synth.py checks that it matches the file.

    python tests/golden/calibrate_synth50_t_end.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle  # noqa: E402
from paper_2312_02836_amd import synth  # noqa: E402

CANDIDATES = [1e-2, 3e-3, 1e-3, 3e-4, 1e-4]
TARGET = 10.0


def main() -> None:
    cfg = synth.config(3, n_cells=4096)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = oracle.OracleNet(spec)
    rows, best = [], None
    for t_end in CANDIDATES:
        _, _, st, cnt = oracle.burn(net, cells, t_end, 1e-6, 1e-10)
        assert np.all(st == 0)
        p5, p50, p95 = np.percentile(cnt[0], [5, 50, 95])
        rows.append((t_end, p5, p50, p95, p95 / p5, cnt[0].mean()))
        if best is None or abs(np.log(p95 / p5 / TARGET)) < abs(np.log(best[4] / TARGET)):
            best = rows[-1]
    with open(os.path.join(HERE, "synth50_t_end.txt"), "w") as f:
        f.write("# 50/150 workload: accepted steps of the oracle on 4,096 seeded cells\n")
        f.write("# (rtol 1e-6, atol 1e-10); written by calibrate_synth50_t_end.py\n")
        f.write("# t_end  p5  p50  p95  p95/p5  mean\n")
        for r in rows:
            f.write(f"# {r[0]:g} {r[1]:.0f} {r[2]:.0f} {r[3]:.0f} {r[4]:.2f} {r[5]:.1f}\n")
        f.write(f"t_end = {best[0]!r}\n")
    print(f"t_end = {best[0]!r} (p95/p5 = {best[4]:.2f})")


if __name__ == "__main__":
    main()
