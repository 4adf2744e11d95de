#!/usr/bin/env python3
"""Benchmark of the low-rank NUFFT hot path on one MI355X; prints one JSON line.

Step (the timed unit): one forward + backward pass of the 1-D type-II
transform through torch.autograd -- f = F2(x) c, loss = ||f - y||^2, then
dL/dc (adjoint kernels) and dL/dx (derivative pass) -- at N = M = 2^22,
complex64, eps = 1e-6, samples iid uniform on [0, 1) (synthetic, seeded).
value = nonuniform points per second through that step (M / step time).

Alongside: per-kernel durations from HIP events recorded by the library on
the launch stream (the roofline of the dominant kernel against 8 TB/s, with
algorithmic bytes = compulsory I/O + one K-wide exchange), the forward
transform alone at N = 2^20 on the fused FP32 path and on the plain FP64
path at the same accuracy (and at eps = 1e-12), and the FP64 direct-sum
oracle timed on the host cores over a bounded sample of rows.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _fail_multi(n):
    print("bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus %d)" % n,
          file=sys.stderr)
    sys.exit(2)


def _progress(msg):
    """One progress line per finished section, on stderr (the JSON line stays alone on stdout)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def kernel_bytes(name, K, N, M, L, cs, ys=None):
    """Algorithmic bytes moved by one launch of a fused kernel: compulsory I/O plus the
    K-wide intermediate written by the first pass and read by the second (ys bytes per
    intermediate value: cs, or 4 for the half-precision exchange)."""
    inter = K * L * (cs if ys is None else ys)
    plan_pts = M * (4 + 4 + 4)           # sorted key, perturbation X (f32), sample index
    table = {
        "fwd_passA": N * cs + inter,
        "fwd_passB": inter + plan_pts + M * cs,
        "gradx_passA": N * cs + inter,
        "gradx_passB": inter + plan_pts + M * cs + M * 8,       # reads sorted g, writes gx (f64)
        "adj_sort": M * cs + M * 4 + M * cs,                    # g, sorted position -> g sorted
        "gradx_sort": M * cs + M * 4 + M * cs,
        "bwd_sort": M * cs + M * 4 + M * cs,
        # large plans: pass B leaves its outputs in the destination-bucketed layout,
        # and this pass moves them to sample order (values, 2-byte in-block index, values)
        "fwd_unsort": M * cs + M * 2 + M * cs,
        "gradx_unsort": M * 8 + M * 2 + M * 8,
        "type1_sort": M * cs + M * 4 + M * cs,
        "adj_passB": M * cs + M * (4 + 4) + (L + 1) * 4 + inter,  # sorted g, X, key, offsets -> Z
        "adj_passA": inter + N * cs,
        "type1_passB": M * cs + M * (4 + 4) + (L + 1) * 4 + inter,
        "type1_passA": inter + N * cs,
    }
    return table.get(name)


def time_loop(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def time_best(fn, steps, warmup, torch, reps=3):
    """Secondary measurements: the best of a few timed loops, so that a pause of the host
    thread (which can leave the GPU idle inside one loop) does not decide the figure."""
    return min(time_loop(fn, steps, warmup if i == 0 else 1, torch) for i in range(reps))


def kernel_source_hash():
    """Hash of every HIP/C++ source the kernels are built from."""
    d = os.path.join(ROOT, "paper_1701_04492_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()[:16]


def traffic_record(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they were
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256_16") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


# Passes that move values between sample order and the destination-bucketed layout:
# not part of the method's compulsory traffic, so the step's algorithmic bytes leave them out.
LAYOUT_PHASES = {"fwd_unsort", "gradx_unsort"}

# Counter runs (rocprofv3 --pmc): the ten kernels of one fwd+bwd step at N = M = 2^22
# in the order the step launches them (the backward sort is two kernels through the
# bucketed layout), then a plain copy of known size whose counters calibrate
# FETCH_SIZE / WRITE_SIZE.
COUNTER_ORDER = ["fwd_passA", "fwd_passB", "fwd_unsort", "bwd_sort.1", "bwd_sort.2", "adj_passB", "adj_passA",
                 "gradx_passA", "gradx_passB", "gradx_unsort"]
COUNTER_KERNELS = ("nufft::k_pass", "nufft::k_bucket_to", "nufft::k_samples_to_bucket")
CALIB_BYTES = 256 << 20


def counter_run(steps):
    import torch
    import paper_1701_04492_amd as P
    from paper_1701_04492_amd import workloads as W
    dev = torch.device("cuda:0")
    N = 1 << 22
    rng = W.rng_for(3)
    c = torch.from_numpy(W.complex_normal(rng, N)).to(torch.complex64).to(dev)
    x = torch.from_numpy(W.iid_samples(rng, N)).to(dev)
    g = torch.from_numpy(W.complex_normal(rng, N)).to(torch.complex64).to(dev)
    # the default grid and schedule (those the step's autotuned plan keeps at this size),
    # without the autotuner's timing launches among the counted dispatches
    plan = P.nufft2_plan(x, N, 1e-6, torch.complex64, P.NUFFT_FLAG_NO_AUTOTUNE)
    f = torch.empty_like(c)
    gc = torch.empty_like(c)
    gx = torch.empty(N, dtype=torch.float64, device=dev)
    assert P.nufft_debug_set_buckets(plan, True), "the 2^22 plan should have the bucketed layout"
    for _ in range(steps):
        P.nufft2_exec(plan, c, f)              # fwd_passA, fwd_passB, fwd_unsort
        P.nufft2_backward(plan, c, g, gc, gx)  # bwd_sort (2 kernels), adj_passB, adj_passA, gradx_passA, _passB, _unsort
    src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)               # calibration: reads and writes CALIB_BYTES
    torch.cuda.synchronize()
    print("counter run done: %d steps, K=%d" % (steps, plan.K), flush=True)


def traffic_summary(fetch_dir, write_dir, out_path, command):
    """rocprofv3 counter CSVs -> HBM bytes per launch of each step kernel."""
    import csv
    import glob

    def read(d, counter):
        rows = []
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(fn)):
                if r["Counter_Name"] == counter:
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        rows.sort()
        lib = [(n, v) for _, n, v in rows if any(k in n for k in COUNTER_KERNELS)]
        cal = [v for _, n, v in rows if "MulFunctor" in n]
        if not cal or not lib or len(lib) % len(COUNTER_ORDER):
            raise SystemExit("unexpected dispatches in %s (%d library, %d calibration)" % (d, len(lib), len(cal)))
        per = {k: [] for k in COUNTER_ORDER}
        names = {}
        for i, (n, v) in enumerate(lib):
            k = COUNTER_ORDER[i % len(COUNTER_ORDER)]
            per[k].append(v)
            names[k] = n.split("(")[0]
        scale = CALIB_BYTES / (cal[-1] * 1024.0)   # true bytes per counted byte
        return {k: sum(v) / len(v) for k, v in per.items()}, scale, names

    fetch, fs, names = read(fetch_dir, "FETCH_SIZE")
    write, ws, _ = read(write_dir, "WRITE_SIZE")
    rec = {"source_sha256_16": kernel_source_hash(), "command": command,
           "calibration": {"copy_bytes_each_way": CALIB_BYTES, "fetch_scale": round(fs, 4),
                           "write_scale": round(ws, 4)},
           "kernels": {}}
    for k in COUNTER_ORDER:
        b = fetch[k] * 1024.0 * fs + write[k] * 1024.0 * ws
        rec["kernels"][k] = {"kernel": names[k], "fetch_kib": round(fetch[k], 1), "write_kib": round(write[k], 1),
                             "bytes_per_launch": int(b)}
    sub = [rec["kernels"][k] for k in ("bwd_sort.1", "bwd_sort.2")]
    rec["kernels"]["bwd_sort"] = {"kernel": " + ".join(r["kernel"] for r in sub),
                                  "fetch_kib": round(sum(r["fetch_kib"] for r in sub), 1),
                                  "write_kib": round(sum(r["write_kib"] for r in sub), 1),
                                  "bytes_per_launch": sum(r["bytes_per_launch"] for r in sub)}
    json.dump(rec, open(out_path, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def cpu_baseline(x, c, N, seconds, f_gpu=None, eps=None):
    """The FP64 direct-sum oracle on a bounded row sample of the same workload.  With the
    GPU's forward output f_gpu (computed from the same c), the rows the oracle summed also
    give the accuracy of the GPU result: returns (baseline, accuracy or None)."""
    import numpy as np
    from oracle import nudft as D
    cores = D.max_threads()
    D.nudft2(x[:cores], c)            # warm-up: thread pool, first touch of c
    rows = 2 * cores
    while True:                       # grow the sample until it takes about `seconds`
        t0 = time.perf_counter()
        ref = D.nudft2(x[:rows], c)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * seconds or rows >= 8192:
            break
        rows = int(min(8192, rows * max(2.0, seconds / max(dt, 1e-3))))
    # the step needs three N-term sums per point: f_j, (F2^H g)_k and the x-derivative
    base = {
        "value": rows / dt / 3.0,
        "unit": "nonuniform pts/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "%d rows of the N=M=2^22 workload, each a direct FP64 compensated sum of 2^22 "
                  "terms (%.1f s); the fwd+bwd step costs 3 such sums per point" % (rows, dt),
    }
    acc = None
    if f_gpu is not None:
        d = f_gpu[:rows].astype(np.complex128) - ref
        M = x.shape[0]
        acc = {"rows": rows,
               "max_err_over_c_l1": float(np.abs(d).max() / np.abs(c).sum()),
               "bound_4eps": 4 * eps,
               # the paper's metric ||f~ - f||_2 / ||c||_2, its sum over j estimated from the rows
               "l2_err_over_c_l2_est": float(np.sqrt(np.mean(np.abs(d) ** 2) * M) / np.linalg.norm(c))}
    return base, acc


def bench_batch(P, W, torch, dev):
    """512 type-II transforms, N_b = round(2^U(8,16)), eps 1e-6 FP32: the autotuned batch
    (three phased launches or one persistent launch; eager and replayed from a HIP graph),
    each launch mode on its own, against 512 separate launches."""
    Ns, xs_np, cs_np = W.batch_case(4)
    Ns = [int(n) for n in Ns]
    xs = [torch.from_numpy(x).to(dev) for x in xs_np]
    cs = [torch.from_numpy(c).to(torch.complex64).to(dev) for c in cs_np]
    fs = [torch.empty(n, dtype=torch.complex64, device=dev) for n in Ns]
    pts = sum(Ns)
    t0 = time.perf_counter()
    plan = P.nufft_batch_plan(Ns, xs, 1e-6, torch.complex64)   # autotuned (the default)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    t_batch = time_best(lambda: P.nufft_batch_exec(plan, cs, fs), 20, 3, torch)
    modes = {}
    for label, fl in (("phased", P.NUFFT_FLAG_NO_AUTOTUNE),
                      ("persistent", P.NUFFT_FLAG_BATCH_PERSISTENT | P.NUFFT_FLAG_NO_AUTOTUNE)):
        pm = P.nufft_batch_plan(Ns, xs, 1e-6, torch.complex64, fl)
        modes[label + "_us"] = round(time_best(lambda: P.nufft_batch_exec(pm, cs, fs), 20, 3, torch) * 1e3, 1)
        del pm
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            P.nufft_batch_exec(plan, cs, fs)
    t_graph = time_best(lambda: g.replay(), 20, 3, torch)
    singles = [P.nufft2_plan(x, n, 1e-6, torch.complex64, P.NUFFT_FLAG_NO_AUTOTUNE) for x, n in zip(xs, Ns)]

    def run_singles():
        for pl, c, f in zip(singles, cs, fs):
            P.nufft2_exec(pl, c, f)
    t_sep = time_loop(run_singles, 5, 1, torch)
    del singles
    plains = [P.nufft2_plan(x, n, 1e-6, torch.complex64, P.NUFFT_FLAG_PLAIN_UNFUSED) for x, n in zip(xs, Ns)]

    def run_plains():
        for pl, c, f in zip(plains, cs, fs):
            P.nufft2_exec(pl, c, f)
    t_plain = time_loop(run_plains, 5, 1, torch)
    del plains
    return {"members": len(Ns), "points": pts, "K_max": plan.K, "autotuned_grid": plan.grid,
            "plan_s": round(plan_s, 2),
            "autotuned_us": round(t_batch * 1e3, 1), "autotuned_pts_per_s": pts / (t_batch * 1e-3),
            "launch_modes": modes,
            "graph_replay_us": round(t_graph * 1e3, 1),
            "separate_fused_launches_us": round(t_sep * 1e3, 1),
            "separate_plain_launches_us": round(t_plain * 1e3, 1),
            "speedup_vs_separate_plain": round(t_plain / t_graph, 2)}


def bench_half(P, torch, x, c, y, N, M, steps, warmup):
    """The same forward+backward step at Table 1's half precision, eps = 2^-10, with the
    half-precision exchange (fp16 intermediate between the two passes)."""
    plan = P.nufft2_plan(x, N, 2.0 ** -10, torch.complex64, P.NUFFT_FLAG_HALF_EXCHANGE)
    xg = x.clone().requires_grad_(True)
    cg = c.clone().requires_grad_(True)

    def step():
        xg.grad = None
        cg.grad = None
        loss = torch.view_as_real(P.nufft2(xg, cg, plan) - y).pow(2).sum()
        loss.backward()

    ms = time_loop(step, steps, warmup, torch)
    P.nufft_plan_profile(plan, 1, reserve=8 * (steps + 1))
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    kern = {}
    for name, (calls, tot) in P.nufft_plan_profile_read(plan).items():
        avg = tot / calls
        by = kernel_bytes(name, plan.K, N, M, plan.grid, 8, ys=4)
        kern[name] = {"avg_us": round(avg * 1e3, 2),
                      "GBs": None if by is None else round(by / (avg * 1e-3) / 1e9, 1)}
    P.nufft_plan_profile(plan, 0)
    return {"eps": 2.0 ** -10, "K": plan.K, "ms_per_step": round(ms, 4), "pts_per_s": M / (ms * 1e-3),
            "kernels": kern}


def oversampling_grids(N):
    """The grids the autotuner tries for N modes: powers of two, 3 * 2^k and 5 * 2^k with
    N <= L <= 2 L0 that have a two-pass split (or are one-pass powers of two)."""
    L0 = 16
    while L0 < N:
        L0 *= 2
    out = []
    for k in range(4, 24):
        for p in (1, 3, 5):
            L = p << k
            if not N <= L <= 2 * L0 or L > 1 << 23:
                continue
            if p > 1 and not any(128 <= (L // p) // q <= 4096 for q in (64, 128, 256, 512)
                                 if q <= (512 if p == 3 else 256)):
                continue
            out.append(L)
    return sorted(set(out))


def bench_oversampling(P, W, torch, dev):
    """Autotuned oversampling (Sec. 2.3): M = 2^22 iid samples, complex64, eps 1e-6, for
    N = 2^14 and N = 20000 modes: the default grid L0 (the power of two >= N), the plan's
    timed choice, and every candidate grid planned explicitly (type II and adjoint)."""
    M = 1 << 22
    rng = W.rng_for(7)
    x = torch.from_numpy(W.iid_samples(rng, M)).to(dev)
    f = torch.empty(M, dtype=torch.complex64, device=dev)
    res = {}
    for N in (1 << 14, 20000):
        c = torch.from_numpy(W.complex_normal(rng, N)).to(torch.complex64).to(dev)
        out = {"N": N, "M": M}

        def timed(pl):
            t = time_best(lambda: P.nufft2_exec(pl, c, f), 20, 3, torch)
            ta = time_best(lambda: P.nufft1_exec(pl, f, +1, c), 10, 2, torch)
            return {"grid": pl.grid, "K": pl.K, "gamma": round(pl.gamma, 4), "us": round(t * 1e3, 2),
                    "pts_per_s": M / (t * 1e-3), "adjoint_us": round(ta * 1e3, 2)}
        for label, fl in (("default", P.NUFFT_FLAG_NO_AUTOTUNE), ("autotuned", 0)):
            pl = P.nufft2_plan(x, N, 1e-6, torch.complex64, fl)
            out[label] = timed(pl)
            del pl
        grids = {}
        for L in oversampling_grids(N):
            pl = P.nufft2_plan(x, N, 1e-6, torch.complex64, P.NUFFT_FLAG_NO_AUTOTUNE, grid=L)
            r = timed(pl)
            grids[str(L)] = {k: r[k] for k in ("K", "us", "adjoint_us")}
            del pl
        out["grids"] = grids
        out["speedup"] = round(out["default"]["us"] / out["autotuned"]["us"], 3)
        res["N%d" % N] = out
    return res


def bench_type3(P, W, torch, dev):
    """Type III (Sec. 3.2), planning included (each call plans its inner transforms):
    1-D with M = N = 2^20, and 2-D with M = Q = 2^16 on 256 x 256 frequency boxes;
    complex64, eps 1e-6, iid samples and frequencies."""
    rng = W.rng_for(8)
    out = {}
    N = 1 << 20
    x = torch.from_numpy(W.iid_samples(rng, N)).to(dev)
    w = torch.from_numpy(rng.uniform(0, N, N)).to(dev)
    c = torch.from_numpy(W.complex_normal(rng, N)).to(torch.complex64).to(dev)
    t = time_loop(lambda: P.nufft3_exec(x, w, c, 1e-6), 5, 1, torch)
    out["1d_2p20"] = {"ms": round(t, 3), "pts_per_s": N / (t * 1e-3)}
    M, n = 1 << 16, 256
    x, y = (torch.from_numpy(W.iid_samples(rng, M)).to(dev) for _ in range(2))
    w1, w2 = (torch.from_numpy(rng.uniform(0, n, M)).to(dev) for _ in range(2))
    c = torch.from_numpy(W.complex_normal(rng, M)).to(torch.complex64).to(dev)
    t = time_loop(lambda: P.nufft2d3_exec(x, y, w1, w2, n, n, c, 1e-6), 3, 1, torch)
    out["2d_2p16_256x256"] = {"ms": round(t, 3), "pts_per_s": M / (t * 1e-3)}
    return out


def bench_3d(P, W, torch, dev):
    """3-D type II and type I, 64^3 modes, M = 2^18 iid samples in [0, 1)^3, complex64, eps 1e-6;
    each call plans (one 2-D plan per z slice) and transforms."""
    rng = W.rng_for(9)
    n, M = 64, 1 << 18
    x, y, z = (torch.from_numpy(W.iid_samples(rng, M)).to(dev) for _ in range(3))
    C = torch.from_numpy(W.complex_normal(rng, n ** 3).reshape(n, n, n)).to(torch.complex64).to(dev)
    t = time_loop(lambda: P.nufft3d_exec(x, y, z, C, 1e-6), 3, 1, torch)
    c = torch.from_numpy(W.complex_normal(rng, M)).to(torch.complex64).to(dev)
    Cout = torch.empty((n, n, n), dtype=torch.complex64, device=dev)
    t1 = time_loop(lambda: P.nufft3d_type1_exec(x, y, z, c, (n, n, n), 1e-6, sign=-1, C=Cout), 3, 1, torch)
    # the reusable plan: built once, then type II / type I calls that only launch kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = P.nufft3d_plan(x, y, z, (n, n, n), 1e-6, torch.complex64)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    f = torch.empty(M, dtype=torch.complex64, device=dev)
    te = time_best(lambda: P.nufft3d_plan_exec(plan, C, f), 10, 2, torch)
    te1 = time_best(lambda: P.nufft3d_plan_type1(plan, c, -1, Cout), 10, 2, torch)
    return {"modes": [n, n, n], "M": M, "K3": plan.K, "ms": round(t, 3), "pts_per_s": M / (t * 1e-3),
            "type1_ms": round(t1, 3),
            "plan": {"plan_ms": round(plan_ms, 3), "type2_exec_ms": round(te, 3), "type1_exec_ms": round(te1, 3),
                     "type2_exec_pts_per_s": M / (te * 1e-3)}}


def bench_solve(P, W, torch, dev):
    """Inverse type II (Sec. 3.3) at N = M = 2^20, complex64, perturbed equispaced samples
    x_j = (j + U(-1/8, 1/8))/N, f = F2 c for c complex N(0,1): CG to a residual of 1e-5."""
    import numpy as np
    N = 1 << 20
    rng = W.rng_for(6)
    x = (np.arange(N) + 0.125 * rng.uniform(-1.0, 1.0, N)) / N
    c = torch.from_numpy(W.complex_normal(rng, N)).to(torch.complex64).to(dev)
    plan = P.nufft2_plan(torch.from_numpy(x).to(dev), N, 1e-6, torch.complex64)
    f = P.nufft2_exec(plan, c)
    P.nufft2_solve(plan, f, tol=1e-5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol, it, res = P.nufft2_solve(plan, f, tol=1e-5)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err = (sol - c).abs().max().item() / c.abs().max().item()
    out = {"N": N, "gamma": 0.125, "iterations": it, "residual": res, "ms": round(dt * 1e3, 2),
           "ms_per_iteration": round(dt * 1e3 / max(it, 1), 3), "max_rel_err_vs_c": err}
    # inverse type I on the same samples: f1 = F1 c, then solve F1 c = f1
    f1 = P.nufft1_exec(plan, c, sign=-1)
    P.nufft1_solve(plan, f1, tol=1e-5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol, it, res = P.nufft1_solve(plan, f1, tol=1e-5)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err = (sol - c).abs().max().item() / c.abs().max().item()
    out["type1"] = {"iterations": it, "residual": res, "ms": round(dt * 1e3, 2),
                    "ms_per_iteration": round(dt * 1e3 / max(it, 1), 3), "max_rel_err_vs_c": err}
    return out


def bench_2d(P, W, torch, dev):
    """2-D type II, adjoint and type I, 1024 x 1024 coefficients, 2^20 polar samples, eps 1e-6 FP32."""
    x, y, C = W.polar_case(5)
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    Ct = torch.from_numpy(C.ravel()).to(torch.complex64).to(dev)
    f = torch.empty(x.shape[0], dtype=torch.complex64, device=dev)
    Co = torch.empty_like(Ct)
    plan = P.nufft2d_plan(xt, yt, 1024, 1024, 1e-6, torch.complex64)
    t_f = time_best(lambda: P.nufft2d_exec(plan, Ct, f, 0), 10, 2, torch)
    t_a = time_best(lambda: P.nufft2d_exec(plan, Co, f, 1), 10, 2, torch)
    t_1 = time_best(lambda: P.nufft2d_type1_exec(plan, f, Co, -1), 10, 2, torch)
    P.nufft_plan_profile(plan, 1, reserve=96)
    for _ in range(5):
        P.nufft2d_exec(plan, Ct, f, 0)
        P.nufft2d_exec(plan, Co, f, 1)
        P.nufft2d_type1_exec(plan, f, Co, -1)
    torch.cuda.synchronize()
    kern = {k: round(ms / n * 1e3, 1) for k, (n, ms) in P.nufft_plan_profile_read(plan).items()}
    P.nufft_plan_profile(plan, 0)
    # algorithmic flops of one direction (the ALU roofline of this ALU/LDS-bound case):
    # Ky length-1024 FFTs per coefficient column (pass A), Kx Ky per grid column (pass B),
    # 5 n log2 n each, plus ~8 flops per sample and rank pair for the gather/spread
    K1 = K2 = plan.K   # gamma -> 1/2 on both axes for the polar samples: Kx = Ky
    n, M = 1024, x.shape[0]
    flop = 5 * n * n * 10 * (K2 + K1 * K2) + 8 * M * K1 * K2
    peak = 157.3e12
    peak_np = 78.6e12   # without packed FP32 instructions (the kernels are compiled with them disabled)
    return {"Kx": plan.K, "forward_us": round(t_f * 1e3, 1), "adjoint_us": round(t_a * 1e3, 1),
            "type1_us": round(t_1 * 1e3, 1), "forward_pts_per_s": x.shape[0] / (t_f * 1e-3),
            "alu_roofline": {"alg_gflop": round(flop / 1e9, 2), "peak_tflops_fp32": 157.3,
                             "forward_frac": round(flop / (t_f * 1e-3) / peak, 4),
                             "adjoint_frac": round(flop / (t_a * 1e-3) / peak, 4),
                             "peak_tflops_fp32_non_packed": 78.6,
                             "forward_frac_non_packed": round(flop / (t_f * 1e-3) / peak_np, 4),
                             "adjoint_frac_non_packed": round(flop / (t_a * 1e-3) / peak_np, 4)},
            "kernels_avg_us": kern}


def autograd_step(P, torch, plan, x, c, y):
    """One forward + backward pass through torch.autograd on the plan: f = F2(x) c,
    loss = ||f - y||^2, dL/dc and dL/dx."""
    xg = x.clone().requires_grad_(True)
    cg = c.clone().requires_grad_(True)

    def step():
        xg.grad = None
        cg.grad = None
        f = P.nufft2(xg, cg, plan)
        loss = torch.view_as_real(f - y).pow(2).sum()
        loss.backward()
    return step, xg, cg


def bench_plain_step(P, torch, x, c, y, N, M, eps, steps, warmup):
    """The spec denominator: the same forward+backward step (N = M = 2^22, eps 1e-6)
    on the plain unfused FP64 path (scale, stand-alone FFT passes, stored U, separate
    gather; spread, FFT passes, weighted sum for the adjoint)."""
    plan = P.nufft2_plan(x, N, eps, torch.complex128, P.NUFFT_FLAG_PLAIN_UNFUSED)
    step, _, _ = autograd_step(P, torch, plan, x, c.to(torch.complex128), y.to(torch.complex128))
    ms = time_loop(step, max(3, steps // 4), 2, torch)
    P.nufft_plan_profile(plan, 1, reserve=32 * (steps + 1))
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    kern = {k: round(t / n * 1e3, 1) for k, (n, t) in P.nufft_plan_profile_read(plan).items()}
    P.nufft_plan_profile(plan, 0)
    out = {"K": plan.K, "ms_per_step": round(ms, 4), "pts_per_s": M / (ms * 1e-3), "kernels_avg_us": kern}
    del plan, step
    return out


def bench_config_rows(P, W, torch, dev):
    """Rows of the remaining workload configurations:
    * N = M = 1024, FP64 plain unfused, eps 1e-12 (a launch-latency case);
    * N = M = 2^20 type II on jittered samples x_j = (j + U(-1/2, 1/2))/N, FP32 eps 1e-6 and FP64 1e-12;
    * N = M = 2^20 type I and adjoint, iid and jittered, FP32 eps 1e-6 and FP64 eps 1e-12."""
    out = {}
    x1, c1 = W.type2_case(1, 1024)
    pl = P.nufft2_plan(torch.from_numpy(x1).to(dev), 1024, 1e-12, torch.complex128, P.NUFFT_FLAG_PLAIN_UNFUSED)
    ct = torch.from_numpy(c1).to(dev)
    ft = torch.empty(1024, dtype=torch.complex128, device=dev)
    t = time_best(lambda: P.nufft2_exec(pl, ct, ft), 50, 10, torch)
    out["n1024_fp64_plain_eps1e-12"] = {"K": pl.K, "us": round(t * 1e3, 2), "pts_per_s": 1024 / (t * 1e-3)}
    del pl
    N = 1 << 20
    for dist in ("iid", "jitter"):
        x, c = W.type2_case(2, N, N, dist)
        xt = torch.from_numpy(x).to(dev)
        for label, dt, e in (("fp32_eps1e-6", torch.complex64, 1e-6), ("fp64_eps1e-12", torch.complex128, 1e-12)):
            pl = P.nufft2_plan(xt, N, e, dt)
            ct = torch.from_numpy(c).to(dt).to(dev)
            ft = torch.empty(N, dtype=dt, device=dev)
            row = {"K": pl.K, "grid": pl.grid}
            if dist == "jitter":
                t = time_best(lambda: P.nufft2_exec(pl, ct, ft), 20, 3, torch)
                row["type2_us"] = round(t * 1e3, 2)
                row["type2_pts_per_s"] = N / (t * 1e-3)
            for sign, nm in ((-1, "type1"), (1, "adjoint")):
                t = time_best(lambda: P.nufft1_exec(pl, ft, sign, ct), 20, 3, torch)
                row[nm + "_us"] = round(t * 1e3, 2)
                row[nm + "_pts_per_s"] = N / (t * 1e-3)
            out["2p20_%s_%s" % (dist, label)] = row
            del pl
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--counter-run", action="store_true",
                    help="launch the step kernels in a fixed order plus a calibration copy (for rocprofv3 --pmc)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from two rocprofv3 counter output folders")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(args.traffic_summary[0], args.traffic_summary[1],
                        os.path.join(ROOT, "profiles", "traffic.json"),
                        ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d <FETCH_DIR> -- "
                         "python3 bench.py --counter-run --steps 3",
                         "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <WRITE_DIR> -- "
                         "python3 bench.py --counter-run --steps 3",
                         "python3 bench.py --traffic-summary <FETCH_DIR> <WRITE_DIR>"])
        return
    if args.counter_run:
        counter_run(args.steps)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        _fail_multi(max(args.gpus, int(os.environ.get("WORLD_SIZE", "1"))))

    import numpy as np
    import torch

    import paper_1701_04492_amd as P
    from paper_1701_04492_amd import workloads as W

    dev = torch.device("cuda:0")
    N = M = 1 << 22
    eps = 1e-6
    rng = W.rng_for(3)
    c_np = W.complex_normal(rng, N)
    x_np = W.iid_samples(rng, M)
    y_np = W.complex_normal(rng, M)
    x = torch.from_numpy(x_np).to(dev)
    c = torch.from_numpy(c_np).to(torch.complex64).to(dev)
    y = torch.from_numpy(y_np).to(torch.complex64).to(dev)
    t0 = time.perf_counter()
    plan = P.nufft2_plan(x, N, eps, torch.complex64)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)
    step, xg, cg = autograd_step(P, torch, plan, x, c, y)
    ms = time_loop(step, args.steps, args.warmup, torch)
    assert xg.grad is not None and cg.grad is not None
    value = M / (ms * 1e-3)
    _progress("2^22 step: %.4f ms" % ms)

    # per-kernel durations: same step, events around every library kernel
    P.nufft_plan_profile(plan, 1, reserve=8 * (args.steps + 1))
    step()
    torch.cuda.synchronize()
    P.nufft_plan_profile(plan, 1)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = P.nufft_plan_profile_read(plan)
    P.nufft_plan_profile(plan, 0)
    kernels = {}
    for name, (calls, tot) in prof.items():
        avg = tot / calls
        by = kernel_bytes(name, plan.K, N, M, plan.grid, 8)
        kernels[name] = {"calls": calls, "avg_us": round(avg * 1e3, 2),
                         "alg_bytes": by, "GBs": None if by is None else round(by / (avg * 1e-3) / 1e9, 1)}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["calls"])
    dk = kernels[dom]
    lib_us = sum(v["avg_us"] * v["calls"] for v in kernels.values()) / args.steps
    step_bytes = sum(v["alg_bytes"] * v["calls"] for k, v in kernels.items()
                     if v["alg_bytes"] and k not in LAYOUT_PHASES) / args.steps
    lib_bytes = step_bytes
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dk["GBs"] / HBM_PEAK_GBS, 4), "traffic": traffic_record(dom),
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_us": dk["avg_us"],
                "all_library_kernels": {"us_per_step": round(lib_us, 2),
                                        "GBs": round(lib_bytes / (lib_us * 1e-6) / 1e9, 1),
                                        "frac": round(lib_bytes / (lib_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
                "step": {"alg_bytes": int(step_bytes), "ms": round(ms, 4),
                         "GBs": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                         "frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                "kernels": kernels}

    out = {
        "metric": "NUFFT-II nonuniform pts/s at eps=1e-6 FP32 vs plain FP64; fwd+bwd %HBM roofline",
        "value": value,
        "unit": "nonuniform pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 arithmetic, fp64 samples and factors)",
        "data": "synthetic (seeded numpy PCG64: c, y complex N(0,1), x iid U[0,1))",
        "config": {"workload": "1-D NUFFT-II forward+backward via autograd (type II, adjoint for dL/dc, "
                               "derivative pass for dL/dx), N=M=2^22, complex64, eps=1e-6, iid x, "
                               "loss ||f-y||^2",
                   "N": N, "M": M, "eps": eps, "K": plan.K, "gamma": plan.gamma, "grid": plan.grid,
                   "schedule": P.nufft_plan_tuning(plan)[0],
                   "plan_ms": round(plan_ms, 1)},
        "roofline": roofline,
    }

    if not args.no_secondary:
        # forward transform alone at N = 2^20: fused FP32 vs plain FP64 at the same eps, and FP64 at 1e-12
        N2 = 1 << 20
        r2 = W.rng_for(2)
        c2 = W.complex_normal(r2, N2)
        x2 = torch.from_numpy(W.iid_samples(r2, N2)).to(dev)
        sec = {}
        for label, dt, e, fl in (("fused_fp32_eps1e-6", torch.complex64, 1e-6, 0),
                                 ("plain_fp64_eps1e-6", torch.complex128, 1e-6, P.NUFFT_FLAG_PLAIN_UNFUSED),
                                 ("fused_fp64_eps1e-12", torch.complex128, 1e-12, 0),
                                 ("plain_fp64_eps1e-12", torch.complex128, 1e-12, P.NUFFT_FLAG_PLAIN_UNFUSED)):
            pl = P.nufft2_plan(x2, N2, e, dt, fl)
            ct = torch.from_numpy(c2).to(dt).to(dev)
            ft = torch.empty(N2, dtype=dt, device=dev)
            t = time_loop(lambda: P.nufft2_exec(pl, ct, ft), 20, 3, torch)
            sec[label] = {"K": pl.K, "us": round(t * 1e3, 2), "pts_per_s": N2 / (t * 1e-3)}
            if label == "fused_fp32_eps1e-6":
                # per-kernel durations of the forward and of the adjoint at this size
                P.nufft_plan_profile(pl, 1, reserve=64)
                for _ in range(10):
                    P.nufft2_exec(pl, ct, ft)
                    P.nufft1_exec(pl, ft, +1, ct)
                torch.cuda.synchronize()
                sec["kernels_fused_fp32"] = {
                    k: {"avg_us": round(ms / n * 1e3, 2),
                        "GBs": round(kernel_bytes(k, pl.K, N2, N2, pl.grid, 8) / (ms / n * 1e-3) / 1e9, 1)}
                    for k, (n, ms) in P.nufft_plan_profile_read(pl).items()}
                P.nufft_plan_profile(pl, 0)
            del pl
        sec["speedup_fused_fp32_vs_plain_fp64_same_eps"] = round(
            sec["plain_fp64_eps1e-6"]["us"] / sec["fused_fp32_eps1e-6"]["us"], 2)
        out["forward_2p20"] = sec
        _progress("2^20 forward rows")

    if not args.no_secondary:
        ps = bench_plain_step(P, torch, x, c, y, N, M, eps, args.steps, args.warmup)
        ps["speedup_fused_fp32_vs_plain_fp64"] = round(ps["ms_per_step"] / ms, 2)
        out["fwd_bwd_2p22_plain_fp64"] = ps
        _progress("fwd_bwd_2p22_plain_fp64")
        out["config_rows"] = bench_config_rows(P, W, torch, dev)
        _progress("config_rows")
        out["fwd_bwd_2p22_half"] = bench_half(P, torch, xg.detach(), c, y, N, M, args.steps, args.warmup)
        _progress("fwd_bwd_2p22_half")
        out["batch_512"] = bench_batch(P, W, torch, dev)
        _progress("batch_512")
        out["polar_2d"] = bench_2d(P, W, torch, dev)
        _progress("polar_2d")
        out["inverse_2p20"] = bench_solve(P, W, torch, dev)
        _progress("inverse_2p20")
        out["oversampling_2p22_samples"] = bench_oversampling(P, W, torch, dev)
        _progress("oversampling_2p22_samples")
        out["type3"] = bench_type3(P, W, torch, dev)
        _progress("type3")
        out["type2_3d"] = bench_3d(P, W, torch, dev)
        _progress("type2_3d")

    if not args.no_cpu_baseline:
        import numpy as np
        f_gpu = P.nufft2_exec(plan, c).cpu().numpy()
        c_in = c.cpu().numpy().astype(np.complex128)   # the complex64 input the GPU transformed
        out["cpu_baseline"], out["accuracy_2p22_forward"] = cpu_baseline(x_np, c_in, N, args.cpu_seconds,
                                                                         f_gpu, eps)
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        _progress("cpu baseline")
    # release every plan and the device tensors before returning
    del plan, step, xg, cg
    import gc
    gc.collect()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
