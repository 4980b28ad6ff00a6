"""Comparison of a GPU burn with the oracle's (shared by the GPU tests and the
smoke check).  Criterion per component: |y_gpu - y_oracle| <= rtol |y_oracle|
+ atol, for every cell; statuses must match exactly."""
from __future__ import annotations

import numpy as np


def stack_state(Y, T):
    return np.vstack([np.asarray(Y), np.asarray(T)[None, :]])


def compare(Yg, Tg, stg, cntg, Yo, To, sto, cnto, rtol, atol):
    yg, yo = stack_state(Yg, Tg), stack_state(Yo, To)
    scale = rtol * np.abs(yo) + atol
    with np.errstate(invalid="ignore", divide="ignore"):
        ewt = np.abs(yg - yo) / scale
    same = (yg == yo) | (np.isnan(yg) & np.isnan(yo))  # also unchanged inf / nan inputs
    ewt = np.where(same, 0.0, np.where(np.isnan(ewt), np.inf, ewt))
    same_cnt = np.all(np.asarray(cntg) == np.asarray(cnto), axis=0)
    per_cell = ewt.max(axis=0) if ewt.size else np.zeros(0)
    return {
        "n_cells": int(yo.shape[1]),
        "status_equal": bool(np.array_equal(np.asarray(stg), np.asarray(sto))),
        "max_ewt": float(per_cell.max()) if per_cell.size else 0.0,
        "n_violations": int((per_cell > 1.0).sum()),
        "violating_cells": np.nonzero(per_cell > 1.0)[0],
        "counter_equal_frac": float(same_cnt.mean()) if same_cnt.size else 1.0,
        "max_ewt_same_counters": float(per_cell[same_cnt].max()) if same_cnt.any() else 0.0,
    }


def summary(rep) -> str:
    return (f"cells={rep['n_cells']} status_equal={rep['status_equal']} "
            f"max_ewt={rep['max_ewt']:.3e} violations={rep['n_violations']} "
            f"counters_equal={rep['counter_equal_frac']:.5f} "
            f"max_ewt(same counters)={rep['max_ewt_same_counters']:.3e}")
