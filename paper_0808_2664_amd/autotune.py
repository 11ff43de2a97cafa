"""Autotuner for the tree shape of batched TSQR.

The block height is fixed by the factor kernel (64 rows); what remains to
choose per matrix is how its rows are split into chains (the flat-tree part
of Sec. 2.1) and the arity of the tree over the chain R factors.  Long chains
keep the tree shallow; short chains expose more parallelism per matrix.  In a
batch the other matrices already supply parallelism, so the best split
depends on the matrix size and column count.

The tuner times candidate policies (rows per chain, arity) on homogeneous
synthetic batches, one per (column class, row bucket), and stores the fastest
in a JSON table keyed by device, dtype, class and bucket.  ``choose`` and
``choose_batch`` read the table (falling back to 4096 rows per chain, binary
tree).  Run ``python -m paper_0808_2664_amd.autotune`` on the target GPU to
(re)build the table.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning.json")

CHAIN_ROWS = (1024, 2048, 4096, 8192, 16384, 65536)
ARITIES = (2, 4)
DEFAULT = {"chain_rows": 4096, "arity": 2}
# row buckets: [2^k, 2^(k+1)) for k = 9..16 (m from 512 to 65536 and above)
BUCKET_LO, BUCKET_HI = 9, 16


def column_class(n: int) -> int:
    return 8 if n <= 8 else 16 if n <= 16 else 32 if n <= 32 else 64


def row_bucket(m: int) -> int:
    k = int(math.floor(math.log2(max(m, 1))))
    return min(max(k, BUCKET_LO), BUCKET_HI)


def _key(device: str, dtype: str, nc: int, bucket: int) -> str:
    return "%s|%s|n%d|m2^%d" % (device, dtype, nc, bucket)


def _dtype_name(dtype) -> str:
    import torch
    return "f64" if dtype == torch.float64 else "f32"


def device_name(device=None) -> str:
    import torch
    props = torch.cuda.get_device_properties(device if device is not None else 0)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


_cache = None


def load_table(path: str = TABLE) -> dict:
    global _cache
    if _cache is None:
        _cache = json.load(open(path)) if os.path.exists(path) else {}
    return _cache


def policy(m: int, n: int, dtype, device: str | None = None) -> dict:
    """(rows per chain, arity) for one matrix, from the table or the default."""
    table = load_table().get("entries", {})
    dev = device or load_table().get("device", "")
    return table.get(_key(dev, _dtype_name(dtype), column_class(n), row_bucket(m)), DEFAULT)


def choose(m: int, n: int, dtype, device: str | None = None):
    p = policy(m, n, dtype, device)
    chains = max(1, -(-m // int(p["chain_rows"])))
    return chains, int(p["arity"])


def choose_batch(shapes, dtype, device: str | None = None):
    return [choose(m, n, dtype, device) for m, n in shapes]


def _time_batch(shapes, dtype, opts, seed: int, reps: int = 3) -> float:
    """Median time (ms) of one batched factorisation of synthetic matrices."""
    import torch
    from .tsqr import BatchPlan
    gen = torch.Generator(device="cuda").manual_seed(seed)
    src = [torch.randn(m, n, dtype=dtype, device="cuda", generator=gen) for m, n in shapes]
    work = [a.clone() for a in src]
    plan = BatchPlan(shapes, dtype=dtype, opts=opts)
    plan.factor(work)  # capture + warm-up
    times = []
    for _ in range(reps):
        for w, s in zip(work, src):
            w.copy_(s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.factor(work)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    plan.close()
    return sorted(times)[len(times) // 2]


def tune(dtype, per_bucket: int = 128, seed: int = 2024, classes=(8, 16, 32, 64), log=print) -> dict:
    """Time every candidate policy on a homogeneous batch per (class, bucket)."""
    import numpy as np
    dev = device_name()
    dname = _dtype_name(dtype)
    entries = {}
    rng = np.random.default_rng(seed)
    for nc in classes:
        for k in range(BUCKET_LO, BUCKET_HI + 1):
            lo, hi = 2 ** k, min(2 ** (k + 1), 65537)
            ms = rng.integers(lo, hi, size=per_bucket)
            ns = rng.integers(max(1, nc // 2 + 1) if nc > 8 else 1, nc + 1, size=per_bucket)
            shapes = [(int(m), int(max(1, min(n, m)))) for m, n in zip(ms, ns)]
            best = None
            for L in CHAIN_ROWS:
                for a in ARITIES:
                    opts = [(max(1, -(-m // L)), a) for m, _ in shapes]
                    t = _time_batch(shapes, dtype, opts, seed + k)
                    if best is None or t < best[0]:
                        best = (t, L, a)
            entries[_key(dev, dname, nc, k)] = {"chain_rows": best[1], "arity": best[2],
                                                "ms_batch": round(best[0], 4), "batch": per_bucket}
            log("%s n<=%d m in [%d,%d): chain_rows %d arity %d  %.3f ms / %d matrices"
                % (dname, nc, lo, hi, best[1], best[2], best[0], per_bucket))
    return {"device": dev, "entries": entries}


def main():
    import torch
    ap = argparse.ArgumentParser(description="tune the batched TSQR tree shapes on this GPU")
    ap.add_argument("--dtype", choices=("f64", "f32", "both"), default="both")
    ap.add_argument("--per-bucket", type=int, default=128)
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args()
    out = {"device": device_name(), "entries": {}}
    if os.path.exists(a.out):
        old = json.load(open(a.out))
        if old.get("device") == out["device"]:
            out["entries"].update(old.get("entries", {}))
    t0 = time.time()
    for d in ((torch.float64, torch.float32) if a.dtype == "both" else
              ((torch.float64,) if a.dtype == "f64" else (torch.float32,))):
        res = tune(d, per_bucket=a.per_bucket, log=lambda s: print(s, flush=True))
        out["entries"].update(res["entries"])
    out["tuned_seconds"] = round(time.time() - t0, 1)
    json.dump(out, open(a.out, "w"), indent=1, sort_keys=True)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
