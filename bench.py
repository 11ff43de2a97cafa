#!/usr/bin/env python3
"""Benchmark of the TSQR hot path on one MI355X.

One step = the whole TSQR pass over the 2^20 x 64 FP64 matrix of the
bandwidth-bound configuration (A = G diag(s) W, cond 1e8; B 2^20 x 32):
    tsqr_factor(A) -> R, implicit Q;  tsqr_apply_qt(B);  tsqr_form_q.
Inputs are resident in HBM before the timed region: every step works on its
own pristine copy of A and B (the factorisation overwrites A), so no copy is
timed and no step reads another step's data out of the caches.

Prints ONE JSON line.  `value` is GFLOP/s of the whole step with the nominal
flop counts of the paper's cost model (factor 2mn^2 - 2n^3/3, Sec. 2.2
Eq. TSQR_seq_runtime; apply Q^T to k columns 4mnk - 2n^2k; explicit Q
2mn^2 - 2n^3/3).  The roofline object is for the dominant kernel (the chain
factor kernel), timed with HIP events on its own stream; its algorithmic
bytes are 2*8*m*n (A read once, reflectors written once: Table 4, 2mn words).

Extra objects on the same line (each also alone with --extra NAME): CAQR of a
16384^2 matrix with FP64 and FP32 updates, the batched plan of 2000 uneven
matrices, forward against forward + backward of the differentiable TSQR,
least squares through TSQR, and TSQR against CholeskyQR / CholeskyQR2.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector / matrix, published
METRIC = "TSQR/CAQR GFLOP/s + HBM GB/s vs roofline; batched & fwd+bwd vs plain"
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_factor_2p20x64_f64.json")
KERNEL_SRC = [os.path.join(ROOT, "paper_0808_2664_amd", "csrc", f)
              for f in ("tsqr_factor.hip", "tsqr_factor_kernel.hpp", "tsqr_wave.hpp", "tsqr_wave2.hpp",
                        "tsqr_common.hpp")]
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector / matrix, published


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--m", type=int, default=1 << 20)
    p.add_argument("--n", type=int, default=64)
    p.add_argument("--k", type=int, default=32)
    p.add_argument("--block-rows", type=int, default=0)
    p.add_argument("--chains", type=int, default=0)
    p.add_argument("--arity", type=int, default=0)
    p.add_argument("--cpu-rows", type=int, default=1 << 19,
                   help="rows of the bounded oracle sample for cpu_baseline (0 = skip)")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the batched, CAQR and forward+backward measurements")
    p.add_argument("--extra", choices=("batched", "caqr", "fwd_bwd", "config1", "lstsq", "cholqr", "caqr_left"),
                   default=None,
                   help="run only this measurement and print its JSON (for profiling it)")
    p.add_argument("--no-oracle", action="store_true",
                   help="with --extra caqr: skip the host oracle's R (for profiling the GPU part alone)")
    p.add_argument("--caqr-reps", type=int, default=10,
                   help="timed CAQR factorisations per update type (median reported)")
    return p.parse_args()


def flops(m, n, k):
    f_factor = 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
    f_apply = 4.0 * m * n * k - 2.0 * n * n * k
    f_formq = 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
    return f_factor, f_apply, f_formq


def bytes_alg(m, n, k, es=8):
    return 2.0 * es * m * n, es * (m * n + 2.0 * m * k), 2.0 * es * m * n


def src_hash(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(m, n):
    """HBM bytes per factor call (the chain kernel and the tree launch) from
    committed rocprofv3 counters (FETCH_SIZE / WRITE_SIZE), scaled by a copy
    kernel of known size; null if absent or taken on another version of the
    kernels."""
    try:
        with open(PMC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != src_hash(KERNEL_SRC):
        return None
    if d.get("m") != m or d.get("n") != n:
        return None
    return d.get("traffic_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(rows, n, k):
    """The oracle (plain C, FP64, pairwise sums) on a bounded sample of the
    step's workload: factor, Q^T B and the explicit Q of the first `rows`
    rows, once with all the host's cores (OpenMP over independent columns)
    and once single-threaded."""
    import oracle
    import workloads
    A = workloads.conditioned(rows, n, 1e8, 2, 3)
    B = workloads.gaussian(rows, k, 4)
    f = sum(flops(rows, n, k))

    def once():
        t0 = time.perf_counter()
        YR, tau = oracle.geqrf(A)
        oracle.apply_qt(YR, tau, B)
        oracle.form_q(YR, tau)
        return time.perf_counter() - t0
    nt = oracle.set_threads(0)
    try:
        dt_all = once()
        oracle.set_threads(1)
        dt_one = once()
    finally:
        oracle.set_threads(nt)
    return {"value": round(f / dt_all / 1e9, 4), "unit": "GFLOP/s", "cores": nt, "kind": "oracle",
            "sample": "factor + apply_qt(k=%d) + form_q on %d x %d FP64 (cond 1e8), C with OpenMP, %d threads, "
                      "%.2f s" % (k, rows, n, nt, dt_all),
            "single_thread": {"value": round(f / dt_one / 1e9, 4), "seconds": round(dt_one, 2)},
            "cpu": cpu_model()}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); "
              "the multi-GPU TSQR is a design note, not built." % a.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if a.extra:
        import paper_0808_2664_amd as tq_x
        fn = {"batched": bench_batched, "caqr": bench_caqr, "fwd_bwd": bench_fwd_bwd, "config1": bench_config1,
              "lstsq": bench_lstsq, "cholqr": bench_cholqr, "caqr_left": bench_caqr_left}[a.extra]
        if a.extra == "caqr":
            res = bench_caqr(tq_x, torch, np, oracle_check=not a.no_oracle, reps=max(1, a.caqr_reps))
        else:
            res = fn(tq_x, torch, np)
        print(json.dumps({a.extra: res}), flush=True)
        return

    import workloads
    import paper_0808_2664_amd as tq
    from paper_0808_2664_amd import _lib

    lib = _lib.load()
    dev = torch.device("cuda:0")
    m, n, k = a.m, a.n, a.k
    extras = {}
    if not a.no_extras:
        # CAQR first (a process's first large allocations and the CU-masked
        # streams it makes), then the TSQR step on the caller's stream
        print("bench: caqr", file=sys.stderr, flush=True)
        extras["caqr"] = bench_caqr(tq, torch, np, reps=max(1, a.caqr_reps))
        extras["caqr"]["schedule"] = "CU split between panels and updates from 8192 (FP64) / 12288 (FP32) trailing columns"
        print("bench: caqr_left", file=sys.stderr, flush=True)
        extras["caqr_left"] = bench_caqr_left(tq, torch, np)
        # CAQR's CU-masked streams and the workspace pool's cached memory are
        # released before the TSQR step (while the masked streams exist, work
        # on the process's other streams ran slower: the step 2.08 against
        # 1.79 ms in one run)
        _lib.check("tsqr_release_streams", lib.tsqr_release_streams())
        _lib.check("tsqr_release_workspace_pools", lib.tsqr_release_workspace_pools())
        torch.cuda.empty_cache()
    print("bench: generating %d x %d (cond 1e8) and %d x %d" % (m, n, m, k), file=sys.stderr, flush=True)
    A_np, B_np = workloads.cfg2(m, n, k)
    A0 = torch.from_numpy(A_np).to(dev)
    B0 = torch.from_numpy(B_np).to(dev)
    total = a.warmup + a.steps
    As = [A0.clone() for _ in range(total)]
    Bs = [B0.clone() for _ in range(total)]
    Q = torch.empty(m, n, dtype=torch.float64, device=dev)
    kw = dict(block_rows=a.block_rows, chains=a.chains, arity=a.arity)
    stream = torch.cuda.current_stream(dev)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # per-step, per-phase events: whole calls and chain kernels
    call_ev = [[(ev(), ev()) for _ in range(3)] for _ in range(total)]
    ker_ev = [[(ev(), ev()) for _ in range(3)] for _ in range(total)]
    for lst in ker_ev:  # torch creates the HIP event on first record
        for pair in lst:
            for e in pair:
                e.record(stream)
    torch.cuda.synchronize()

    def step(i):
        phases = {0: 0, 1: 1, 2: 3}  # factor, apply_qt, form_q -> library phase ids
        for p, lp in phases.items():
            s, e = ker_ev[i][p]
            lib.tsqr_set_phase_events(lp, ctypes_ptr(s), ctypes_ptr(e))
        c = call_ev[i]
        c[0][0].record(stream)
        R, qt = tq.factor(As[i], **kw)
        c[0][1].record(stream)
        c[1][0].record(stream)
        qt.apply_qt(Bs[i])
        c[1][1].record(stream)
        c[2][0].record(stream)
        qt.form_q(Q)
        c[2][1].record(stream)
        return R, qt

    for i in range(a.warmup):
        R, qt = step(i)
        qt.close()
    torch.cuda.synchronize()
    print("bench: timing %d steps" % a.steps, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for i in range(a.warmup, total):
        R, qt = step(i)
        info = qt.info()
        qt.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for lp in (0, 1, 3):
        lib.tsqr_set_phase_events(lp, None, None)
    ms = (t1 - t0) * 1e3 / a.steps

    def avg(evs, p):
        return sum(evs[i][p][0].elapsed_time(evs[i][p][1]) for i in range(a.warmup, total)) / a.steps

    call_ms = [avg(call_ev, p) for p in range(3)]
    ker_ms = [avg(ker_ev, p) for p in range(3)]
    fl = flops(m, n, k)
    by = bytes_alg(m, n, k)
    value = sum(fl) / (ms / 1e3) / 1e9

    # correctness of the last step (reported on every run)
    tq.sign_normalize(Q, R)
    Rn = R
    res = (torch.linalg.norm(A0 - Q @ Rn) / torch.linalg.norm(A0)).item()
    Qc = Q.reshape(-1, 1024, n)
    G = torch.bmm(Qc.transpose(1, 2).contiguous(), Qc)
    while G.shape[0] > 1:
        G = G[0::2] + G[1::2]
    orth = torch.linalg.norm(G[0] - torch.eye(n, dtype=torch.float64, device=dev)).item()

    dom_ms = ker_ms[0]
    achieved = by[0] / (dom_ms / 1e3) / 1e9
    traffic = traffic_from_profile(m, n)
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "TSQR factor: k_chain2 (two-wave chains) + k_wave_tsqr (pipelined tree), two launches",
            "kernel_ms": round(dom_ms, 4), "algorithmic_bytes": by[0]}
    cpu = None
    if a.cpu_rows > 0:
        print("bench: oracle cpu baseline on %d rows" % a.cpu_rows, file=sys.stderr, flush=True)
        cpu = cpu_baseline(min(a.cpu_rows, m), n, k)
    if not a.no_extras:
        for name, fn in (("batched", bench_batched), ("fwd_bwd", bench_fwd_bwd),
                         ("config1", bench_config1), ("lstsq", bench_lstsq), ("cholqr", bench_cholqr)):
            print("bench: %s" % name, file=sys.stderr, flush=True)
            extras[name] = fn(tq, torch, np)
            torch.cuda.empty_cache()
    names = ("factor", "apply_qt", "form_q")
    phases = {}
    for p, nm in enumerate(names):
        phases[nm] = {"call_ms": round(call_ms[p], 4), "chain_kernel_ms": round(ker_ms[p], 4),
                      "gflops": round(fl[p] / (call_ms[p] / 1e3) / 1e9, 1),
                      "alg_gbs": round(by[p] / (call_ms[p] / 1e3) / 1e9, 1)}
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "TSQR factor + apply_qt + form_q, %d x %d FP64, cond 1e8, B %d x %d" % (m, n, m, k),
                   "m": m, "n": n, "k": k, "block_rows": info["block_rows"], "chains": info["chains"],
                   "arity": info["arity"], "tree_levels": info["levels"], "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "phases": phases,
        "hbm_gbs_step": round(sum(by) / (ms / 1e3) / 1e9, 1),
        "residual": res,
        "orthogonality": orth,
        "host": {"cpu": cpu_model(), "nproc": os.cpu_count()},
    }
    out.update(extras)
    print(json.dumps(out))


def _ev_ms(torch, fn, reps):
    """Median over reps of fn() timed with events on the current stream."""
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return sorted(ts)[len(ts) // 2]


def bench_batched(tq, torch, np):
    """Config 4: 2000 matrices, m ~ U{512..65536}, n in {8,16,32,64}, one graph
    launch with autotuned tree shapes, against 2000 sequential tsqr_factor
    calls (both produce R and the leaf reflectors, no implicit Q); FP64 and
    FP32.  Inputs are drawn on the device (seed 6)."""
    import oracle
    import workloads
    from paper_0808_2664_amd import autotune
    shapes = workloads.cfg4_shapes()
    res = {"workload": "2000 matrices, m ~ U{512..65536}, n in {8,16,32,64}, iid N(0,1) (seed 6)"}
    for dt, name, es in ((torch.float64, "f64", 8), (torch.float32, "f32", 4)):
        src = [workloads.cfg4_device_matrix(i, m, n, dtype=dt) for i, (m, n) in enumerate(shapes)]
        work = [x.clone() for x in src]
        alg = sum(2.0 * es * m * n for m, n in shapes)
        plan = tq.BatchPlan(shapes, dt, opts=autotune.choose_batch(shapes, dt))
        Rs = plan.factor(work)
        torch.cuda.synchronize()

        def run_batched():
            plan.factor(work)

        def reset():
            for w, x in zip(work, src):
                w.copy_(x)
        ts = []
        for _ in range(5):
            reset()
            torch.cuda.synchronize()
            ts.append(_ev_ms(torch, run_batched, 1))
        t_b = sorted(ts)[len(ts) // 2]
        reset()
        torch.cuda.synchronize()

        def run_seq():
            # the same work as the batch: R and the leaf reflectors, no implicit Q
            for w in work:
                tq.factor(w, want_q=False)
        tss = []
        for _ in range(3):
            reset()
            torch.cuda.synchronize()
            tss.append(_ev_ms(torch, run_seq, 1))
        t_s = sorted(tss)[1]
        # worst R error against the oracle on a sample (smallest, largest, an n = 64 one)
        reset()
        Rs = plan.factor(work)
        torch.cuda.synchronize()
        ms_ = np.array([m for m, _ in shapes])
        sample = sorted({int(ms_.argmin()), int(ms_.argmax()), next(i for i, s in enumerate(shapes) if s[1] == 64)})
        worst = 0.0
        for i in sample:
            R = Rs[i].double().cpu().numpy()
            Ro = oracle.qr(src[i].double().cpu().numpy())[1]
            worst = max(worst, oracle.rel_err(R * oracle.signs(R)[:, None], Ro))
        gbs = alg / (t_b / 1e3) / 1e9
        res[name] = {"ms": round(t_b, 3), "runs": len(ts), "alg_gbs": round(gbs, 1),
                     "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "sequential_ms": round(t_s, 3),
                     "sequential_runs": len(tss), "speedup_vs_sequential": round(t_s / t_b, 2),
                     "worst_sampled_R_error": worst, "sample": sample, "plan": plan.info()}
        plan.close()
        del src, work
        torch.cuda.empty_cache()
    return res


def bench_caqr(tq, torch, np, oracle_check=True, reps=10):
    """Config 3: CAQR of a 16384 x 16384 N(0,1) matrix (seed 5, drawn with
    numpy on the host and copied to the device once), panel 64, trailing
    updates in FP64 and with FP32 products on FP64 storage.  Time: median of
    `reps` factorisations each (10 unless --caqr-reps; each on a fresh copy of
    A, after one untimed factorisation).  Errors per result:
    backward error ||A - QR||/||A|| through the GPU's implicit Q, and the
    normwise error of the sign-normalised R against the oracle's blocked
    Householder QR of the same matrix (run on the host after the timings)."""
    import oracle
    import workloads
    N = 16384
    A_np = workloads.cfg3(N)
    A0 = torch.from_numpy(A_np).cuda()
    fl = 4.0 * N ** 3 / 3.0
    res = {"workload": "CAQR 16384 x 16384 FP64 storage, panel 64, N(0,1) seed 5", "flops": fl}
    Rkeep = {}
    for name, upd, peak in (("f64_update", torch.float64, FP64_PEAK_TFLOPS), ("f32_update", torch.float32,
                                                                               FP32_PEAK_TFLOPS)):
        A = A0.clone()
        box = {}

        def run():
            A.copy_(A0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            box["R"], box["qt"] = tq.caqr(A, panel=64, update=upd)
            e1.record()
            torch.cuda.synchronize()
            box["ms"] = e0.elapsed_time(e1)
        run()
        box["qt"].close()
        ts = []
        for r in range(reps):
            run()
            ts.append(box["ms"])
            if r + 1 < reps:
                box["qt"].close()
        ts.sort()
        ms = ts[len(ts) // 2]
        R, qt = box["R"], box["qt"]
        X = torch.zeros(N, N, dtype=torch.float64, device="cuda")
        X.copy_(torch.triu(R))
        qt.apply_q(X)
        be = (torch.linalg.norm(X - A0) / torch.linalg.norm(A0)).item()
        qt.close()
        del X
        tfl = fl / (ms / 1e3) / 1e12
        res[name] = {"ms": round(ms, 2), "ms_min_max": [round(ts[0], 2), round(ts[-1], 2)], "runs": reps,
                     "tflops": round(tfl, 2), "frac_peak": round(tfl / peak, 4), "peak_tflops": peak,
                     "backward_error": be}
        Rkeep[name] = R.cpu().numpy()
        del A, R
        torch.cuda.empty_cache()
    del A0
    torch.cuda.empty_cache()
    if oracle_check:
        print("bench: caqr oracle (blocked Householder QR on the host)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        threads = oracle.set_threads(0)
        YR, _ = oracle.geqrf_blocked(A_np, 64)
        Ro = oracle.r_of(YR)
        del YR
        Ro *= oracle.signs(Ro)[:, None]
        for name, R in Rkeep.items():
            res[name]["R_error_vs_oracle"] = oracle.rel_err(R * oracle.signs(R)[:, None], Ro)
        res["oracle"] = {"kind": "blocked Householder QR, panels of 64, FP64", "threads": threads,
                         "seconds": round(time.perf_counter() - t0, 1)}
    return res


def bench_caqr_left(tq, torch, np):
    """Left-looking CAQR over column blocks (Sec. 3.2), FP64 update, panel
    64: on the 16384^2 N(0,1) matrix of the CAQR measurement (seed 5) with
    blocks of 1024, 4096 and 16384 columns, and plain left-looking (blocks of
    one panel) on a 4096^2 N(0,1) matrix (seed 11) beside right-looking CAQR
    of the same matrix.  Median of 3 factorisations each (after one untimed);
    per result the backward error through the GPU's implicit Q and the
    normwise difference of the sign-normalised R from right-looking CAQR's
    (the oracle comparison is in the GPU tests)."""
    import workloads
    res = {"workload": "left-looking CAQR over column blocks, FP64 storage and update, panel 64", "runs": 3}

    def signed(R):
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1
        return R * d[:, None]

    def timed(A0, fn):
        A = A0.clone()
        ts = []
        for r in range(4):
            A.copy_(A0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            R, qt = fn(A)
            e1.record()
            torch.cuda.synchronize()
            if r > 0:
                ts.append(e0.elapsed_time(e1))
            if r < 3:
                qt.close()
        ts.sort()
        N = A0.shape[1]
        X = torch.zeros_like(A0)
        X[:N] = torch.triu(R)
        qt.apply_q(X)
        be = (torch.linalg.norm(X - A0) / torch.linalg.norm(A0)).item()
        qt.close()
        del X, A
        torch.cuda.empty_cache()
        return ts[len(ts) // 2], signed(R), be

    for N, seed, blocks in ((16384, None, (1024, 4096, 16384)), (4096, 11, (64,))):
        A_np = workloads.cfg3(N) if seed is None else workloads.gaussian(N, N, seed)
        A0 = torch.from_numpy(A_np).cuda()
        del A_np
        fl = 4.0 * N ** 3 / 3.0
        ms_r, R_r, be_r = timed(A0, lambda A: tq.caqr(A, panel=64, update=torch.float64))
        row = {"right_looking": {"ms": round(ms_r, 2), "tflops": round(fl / ms_r / 1e9, 2), "backward_error": be_r}}
        for w in blocks:
            print("bench: caqr_left %d^2 blocks of %d" % (N, w), file=sys.stderr, flush=True)
            ms, R, be = timed(A0, lambda A: tq.caqr_left(A, panel=64, block_cols=w, update=torch.float64))
            dr = (torch.linalg.norm(R - R_r) / torch.linalg.norm(R_r)).item()
            row["block_%d" % w] = {"ms": round(ms, 2), "tflops": round(fl / ms / 1e9, 2), "backward_error": be,
                                   "R_diff_vs_right_looking": dr}
            del R
        res["%dx%d" % (N, N)] = row
        del A0, R_r
        torch.cuda.empty_cache()
    return res


def bench_fwd_bwd(tq, torch, np):
    """Config 5: differentiable TSQR, forward alone against forward +
    backward, on 262144 x 32 FP64 (seed 7; dQ, dR seeds 8, 9) and on the
    FP32 batch of 256 matrices of 8192 x 32 (seed 10; one batched
    factorisation, each member on its own tree, then one explicit-Q pass and
    the batched adjoint)."""
    import workloads
    res = {"workload": "TSQR forward (factor + Q) and backward (QR adjoint): 262144 x 32 FP64; "
                       "batch of 256 x 8192 x 32 FP32"}
    A_np, dQ_np, dR_np = workloads.cfg5()
    Ab_np, dQb_np, dRb_np = workloads.cfg5_batch()
    for name, (a_np, dq_np, dr_np), es in (("f64", (A_np, dQ_np, dR_np), 8), ("f32_batch", (Ab_np, dQb_np, dRb_np), 4)):
        A = torch.from_numpy(a_np).cuda()
        dQ = torch.from_numpy(dq_np).cuda()
        dR = torch.from_numpy(dr_np).cuda()

        def fwd():
            tq.tsqr(A)

        Ag = A.clone().requires_grad_(True)

        def fwd_bwd():
            Ag.grad = None  # each call computes dA afresh (no accumulation into the last call's)
            Q, R = tq.tsqr(Ag)
            torch.autograd.backward((Q, R), (dQ, dR))
        for f in (fwd, fwd_bwd):
            f()
        # host launch gaps are a visible part of each call: median of many calls
        t_f = _ev_ms(torch, fwd, 21)
        t_fb = _ev_ms(torch, fwd_bwd, 21)
        elems = float(A.numel())
        # HBM words: forward reads A, writes Y, reads Y, writes Q; backward reads Q, dQ, writes dA (+ R, dR)
        fb_bytes = es * elems * (4 + 3)
        res[name] = {"shape": list(A.shape), "fwd_ms": round(t_f, 4), "fwd_bwd_ms": round(t_fb, 4),
                     "ratio": round(t_fb / t_f, 3), "fwd_bwd_alg_gbs": round(fb_bytes / (t_fb / 1e3) / 1e9, 1)}
        del A, dQ, dR, Ag
        torch.cuda.empty_cache()
    return res


def bench_config1(tq, torch, np):
    """Config 1: TSQR of one 4096 x 16 FP64 matrix (seed 1), leaves of 256
    rows (16 chains, binary tree), R and the explicit Q: microseconds per
    call (median of 200).  At this size the call is bound by launch and
    synchronisation latency, not by HBM or arithmetic, so no roofline
    fraction is given."""
    import workloads
    A0 = torch.from_numpy(workloads.cfg1()).cuda()
    A = A0.clone()
    Q = torch.empty_like(A0)

    def call():
        A.copy_(A0)
        R, qt = tq.factor(A, chains=16)
        qt.form_q(Q)
        qt.close()

    def copy_only():
        A.copy_(A0)
    for _ in range(5):
        call()
    t = _ev_ms(torch, call, 200)
    t0 = _ev_ms(torch, copy_only, 200)
    return {"workload": "TSQR 4096 x 16 FP64, 16 chains of 256 rows, factor + form_q", "us_per_call": round(1e3 * (t - t0), 2),
            "us_per_call_with_copy": round(1e3 * t, 2)}


def bench_lstsq(tq, torch, np):
    """Least squares through TSQR (factor, Q^T B, back substitution, residual
    norms) on the step's inputs: 2^20 x 64 FP64 (cond 1e8, seeds 2, 3) with
    32 right-hand sides (seed 4); the library call alone, on buffers
    refilled from pristine copies before each call."""
    import ctypes

    import workloads
    from paper_0808_2664_amd import _lib
    A_np, B_np = workloads.cfg2()
    A0 = torch.from_numpy(A_np).cuda()
    B0 = torch.from_numpy(B_np).cuda()
    del A_np, B_np
    m, n = A0.shape
    k = B0.shape[1]
    W, Bw = A0.clone(), B0.clone()
    rn = torch.empty(k, dtype=torch.float64, device="cuda")
    lib = _lib.load()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call():
        rc = lib.tsqr_lstsq(_lib.TSQR_F64, m, n, ctypes.c_void_p(W.data_ptr()), n, k,
                            ctypes.c_void_p(Bw.data_ptr()), k, ctypes.c_void_p(rn.data_ptr()), None, st)
        _lib.check("tsqr_lstsq", rc)
    ts = []
    for it in range(13):
        W.copy_(A0)
        Bw.copy_(B0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        torch.cuda.synchronize()
        if it >= 3:
            ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[len(ts) // 2]
    # nominal counts: factor 2mn^2 - 2n^3/3, Q^T B 4mnk - 2n^2k, solve n^2 k
    fl = 2.0 * m * n * n - 2.0 * n ** 3 / 3 + 4.0 * m * n * k - 2.0 * n * n * k + n * n * k
    # words: read A, write the reflectors, read them again, read and write B
    by = 8.0 * (3 * m * n + 2 * m * k)
    # residual check in FP64 on the device: ||A X - B|| per column against rnorm
    X = Bw[:n]
    rr = torch.linalg.norm(A0 @ X - B0, dim=0)
    return {"workload": "least squares, 1048576 x 64 FP64 (cond 1e8), 32 right-hand sides",
            "ms": round(ms, 4), "gflops": round(fl / (ms / 1e3) / 1e9, 1),
            "alg_gbs": round(by / (ms / 1e3) / 1e9, 1),
            "rnorm_vs_residual": float(torch.max(torch.abs(rr - rn) / rr))}


def bench_cholqr(tq, torch, np):
    """TSQR against CholeskyQR, CholeskyQR2 and modified Gram-Schmidt (the
    comparison of Sec. 2.3) on 2^20 x 64 FP64: the step's matrix (cond 1e8,
    seeds 2, 3) and a Gaussian one (seed 2).  TSQR = factor + form Q on a
    copy refilled before each call; CholeskyQR and MGS read A and write Q.
    Median of 10 calls each, with the orthogonality ||Q^T Q - I||_F of the
    result (null where the Cholesky factorisation broke down)."""
    import workloads
    out = {"workload": "TSQR vs CholeskyQR / CholeskyQR2 / MGS, 1048576 x 64 FP64"}
    for name, A_np in (("cond_1e8", workloads.conditioned(1 << 20, 64, 1e8, 2, 3)),
                       ("gaussian", workloads.gaussian(1 << 20, 64, 2))):
        A0 = torch.from_numpy(A_np).cuda()
        del A_np
        W = A0.clone()
        Q = torch.empty_like(A0)

        def orth(Qx):
            if not bool(torch.isfinite(Qx).all()):
                return None
            G = Qx.T.contiguous() @ Qx
            return float(torch.linalg.norm(G - torch.eye(G.shape[0], dtype=G.dtype, device=G.device)))

        def timed(fn, pre=None):
            ts = []
            for it in range(13):
                if pre is not None:
                    pre()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                if it >= 3:
                    ts.append(e0.elapsed_time(e1))
            return sorted(ts)[len(ts) // 2]
        box = {}

        def tsqr_call():
            _, qt = tq.factor(W)
            qt.form_q(out=Q)
            box["qt"] = qt

        def tsqr_pre():
            if "qt" in box:
                box.pop("qt").close()
            W.copy_(A0)
        res = {"tsqr_ms": round(timed(tsqr_call, tsqr_pre), 4), "tsqr_orthogonality": orth(Q)}
        box.pop("qt").close()
        for passes, key in ((1, "cholqr"), (2, "cholqr2")):
            res[key + "_ms"] = round(timed(lambda: tq.cholqr(A0, passes, out_q=Q)), 4)
            res[key + "_orthogonality"] = orth(Q)
        res["mgs_ms"] = round(timed(lambda: tq.mgs(A0, out_q=Q)), 4)
        res["mgs_orthogonality"] = orth(Q)
        out[name] = res
        del A0, W, Q
        torch.cuda.empty_cache()
    return out


def ctypes_ptr(event):
    import ctypes
    return ctypes.c_void_p(event.cuda_event)


if __name__ == "__main__":
    main()
