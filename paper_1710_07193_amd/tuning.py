"""Autotuning table of the library: measure, persist as JSON, re-apply.

The table maps (kernel, block size N, precision) to the launch choice the
library should make on this GPU:

  "batch/N8/<prec>"  : batch plan configuration (fronts, io, nt, groups_per_cu)
                       for plans of N = 8 jobs, chosen by dctf_batch_autotune
  "filter/N<N>/<prec>": single-operator kernel variant (by name), chosen by
                       dctf_autotune

with <prec> "split-bf16" or "fp32".  Every choice computes bit-identical
results; only the time differs.  The workloads timed are sized like the
benchmark's (N = 8: 64 jobs of 65,536 blocks over 16 operators, and a single
operator over 4,194,304 blocks; N = 16: 1,036,800 blocks).  Timing does not
depend on the coefficient values, so the inputs are random.

  python -m paper_1710_07193_amd.tuning            # measure and write the table
  apply_table()                                    # load it and set the library
"""
from __future__ import annotations

import datetime
import json
import os
import sys

import numpy as np
import torch

from . import (DCTF_PREC_FP32, DCTF_PREC_SPLIT_BF16, DCTF_RUN_REBUILD_OPERATORS, dctf_autotune,
               dctf_batch_autotune, dctf_batch_create, dctf_batch_get_config, dctf_build_operator,
               dctf_build_operators, dctf_set_batch_config, dctf_set_variant, dctf_variant_count,
               dctf_variant_name, dctf_version)

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")
PREC_NAMES = {DCTF_PREC_SPLIT_BF16: "split-bf16", DCTF_PREC_FP32: "fp32"}
PREC_OF = {v: k for k, v in PREC_NAMES.items()}


def key(kernel: str, N: int, prec: int) -> str:
    return "%s/N%d/%s" % (kernel, N, PREC_NAMES[prec])


def _random_masks(count: int, seed: int):
    """Sum-1 masks of sizes 3, 5, 7 (the values do not change the timing)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        k = (3, 5, 7)[i % 3]
        W = rng.uniform(0.0, 1.0, size=(k, k))
        out.append(W / W.sum())
    return out


def tune_batch(prec: int, images: int = 64, blocks: int = 65536, masks: int = 16, iters: int = 10,
               rounds: int = 3, seed: int = 11) -> dict:
    """Tune the batch plan of `images` jobs of `blocks` 8x8 blocks each (one
    of `masks` operators per job, border replication), as one step with the
    operator rebuild."""
    ops = dctf_build_operators([(W, 8, 1) for W in _random_masks(masks, seed)])
    X = torch.randn(images * blocks * 64, device="cuda") * 100.0
    Y = torch.empty_like(X)
    per = blocks * 64
    draws = np.random.default_rng(seed).integers(0, masks, size=images)
    jobs = [(ops[draws[i]], X[i * per:(i + 1) * per], Y[i * per:(i + 1) * per]) for i in range(images)]
    batch = dctf_batch_create(jobs, prec)
    best, table = dctf_batch_autotune(batch, DCTF_RUN_REBUILD_OPERATORS, iters, rounds)
    cfg, resolved = dctf_batch_get_config(batch)
    ms = table[best][1]
    return {"config": cfg, "resolved": resolved, "ms_per_launch": ms,
            "workload": "%d jobs x %d blocks of 8x8, %d operators, one step = operator rebuild + launch"
                        % (images, blocks, masks),
            "candidates": [dict(c, ms=t) for c, t in table]}


def tune_filter(N: int, prec: int, blocks: int, iters: int = 10, seed: int = 12) -> dict:
    """Tune the single-operator kernel variant of block size N."""
    op = dctf_build_operator(_random_masks(1, seed)[0], N, 0)
    X = torch.randn(blocks * N * N, device="cuda") * 100.0
    Y = torch.empty_like(X)
    best, ms = dctf_autotune(op, prec, X, Y, iters)
    return {"variant": dctf_variant_name(N, prec, best), "ms_per_launch": ms,
            "workload": "%d blocks of %dx%d, one operator" % (blocks, N, N)}


def tune_all() -> dict:
    table = {"device": torch.cuda.get_device_name(0), "library": dctf_version(),
             "date": datetime.date.today().isoformat(), "entries": {}}
    e = table["entries"]
    for prec in (DCTF_PREC_SPLIT_BF16, DCTF_PREC_FP32):
        e[key("batch", 8, prec)] = tune_batch(prec)
        print("tuned", key("batch", 8, prec), e[key("batch", 8, prec)]["config"],
              "%.4f ms" % e[key("batch", 8, prec)]["ms_per_launch"], flush=True)
        for N, blocks in ((8, 4194304), (16, 1036800)):
            e[key("filter", N, prec)] = tune_filter(N, prec, blocks)
            print("tuned", key("filter", N, prec), e[key("filter", N, prec)]["variant"], flush=True)
    return table


def save(table: dict, path: str = TABLE_PATH):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)


def load(path: str = TABLE_PATH):
    """The persisted table, or None if there is none."""
    try:
        with open(path) as f:
            return json.load(f)
    except OSError:
        return None


def validate(table: dict):
    """Checks every entry names a known key, variant and configuration range
    (no GPU needed).  Raises ValueError."""
    for k, v in table.get("entries", {}).items():
        kernel, n, pname = k.split("/")
        N = int(n[1:])
        if pname not in PREC_OF or kernel not in ("batch", "filter"):
            raise ValueError("unknown table key %r" % k)
        prec = PREC_OF[pname]
        if kernel == "batch":
            c = v["config"]
            if N != 8 or set(c) != {"fronts", "io", "nt", "groups_per_cu"}:
                raise ValueError("bad batch entry %r" % k)
            if not (-1 <= c["fronts"] <= 4096 and -1 <= c["io"] <= 2 and c["nt"] in (0, 1)
                    and 0 <= c["groups_per_cu"] <= 64):
                raise ValueError("batch configuration out of range in %r" % k)
        else:
            names = [dctf_variant_name(N, prec, i) for i in range(dctf_variant_count(N, prec))]
            if v["variant"] not in names:
                raise ValueError("unknown variant %r in %r" % (v["variant"], k))


def apply(table: dict) -> dict:
    """Sets the library to the table's choices; returns the entries applied
    (key -> choice)."""
    validate(table)
    applied = {}
    for k, v in table.get("entries", {}).items():
        kernel, n, pname = k.split("/")
        N, prec = int(n[1:]), PREC_OF[pname]
        if kernel == "batch":
            dctf_set_batch_config(prec, v["config"])
            applied[k] = dict(v["config"])
        else:
            names = [dctf_variant_name(N, prec, i) for i in range(dctf_variant_count(N, prec))]
            dctf_set_variant(N, prec, names.index(v["variant"]))
            applied[k] = v["variant"]
    return applied


def apply_table(path: str = TABLE_PATH):
    """Loads the persisted table and applies it; None if there is none."""
    table = load(path)
    if table is None:
        return None
    return {"source": os.path.basename(path), "device": table.get("device"), "date": table.get("date"),
            "applied": apply(table)}


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    path = argv[0] if argv else TABLE_PATH
    assert torch.cuda.is_available(), "tuning needs the GPU"
    table = tune_all()
    save(table, path)
    print("wrote", path)


if __name__ == "__main__":
    main()
