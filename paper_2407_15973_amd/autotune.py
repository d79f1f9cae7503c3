"""Autotuner of the batched multi-right-hand-side launches.

The batched kernels cut every system into chunks of rows (SpMV) and of whole
blocks (application) and spread the chunks over persistent workgroups. Four
knobs set the shape: ``spmv_grab`` (matrix-vector chunks a wave takes per
grab of its XCD's counter: fewer atomics against a wider window of rows in
flight), ``wg_per_cu`` (workgroups per compute unit of the application),
``spmv_wg_per_cu`` (the same for the matrix-vector product) and
``apply_rows`` (padded rows per apply chunk: fewer partial dot products
against a finer load balance). ``pcg_batched_tune`` in the library times a
few PCG iterations of the actual batch under each candidate; this module
picks the candidates, keys the result by the batch's shape and keeps it in a
JSON cache so a batch of the same shape is not tuned twice.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import binding as mb

CANDIDATES = tuple((g, w, sw, ar) for g in (4, 8) for w in (8, 32) for sw in (3, 32) for ar in (256, 512))


def default_cache_path() -> str:
    return os.environ.get("MPBJAC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mpbjac", "batched_tune.json"))


def shape_key(bs: "mb.BatchSolver") -> str:
    """Batch shape, coarsened to powers of two so nearby shapes share an entry:
    systems, rows, columns, non-zeros and the stored bytes of the map."""
    rows = np.diff(bs.sys_row).astype(np.int64)
    info = bs.M.info()

    def p2(v):
        return int(2 ** round(math.log2(max(1, v))))

    return (f"S{p2(bs.nsys)}-n{p2(int(rows.sum()))}-c{p2(bs.ncols)}-v{p2(bs.veclen)}"
            f"-z{p2(bs.A.nnz)}-m{p2(info['low_bytes'])}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # an unwritable cache only costs a re-tune


def tuned_cfg(bs: "mb.BatchSolver", b, candidates=CANDIDATES, iters=6, cache_path=None, force=False):
    """(spmv_grab, wg_per_cu, spmv_wg_per_cu, apply_rows) for this batch: from the cache, else timed."""
    path = cache_path or default_cache_path()
    key = shape_key(bs)
    data = _load(path)
    if not force and key in data:
        return tuple(data[key]["cfg"]), data[key]
    best, ms = bs.tune(b, list(candidates), iters=iters)
    entry = {"cfg": list(candidates[best]),
             "ms_per_iter": {"x".join(str(v) for v in c): float(t) for c, t in zip(candidates, ms)}}
    data[key] = entry
    _save(path, data)
    return tuple(candidates[best]), entry
