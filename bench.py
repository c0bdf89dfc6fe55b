#!/usr/bin/env python3
"""Throughput of randomized Cholesky QR (Balabanov, arXiv 2210.09953) on one
MI355X: GB/s of X factored and ||Q^T Q - I||_2, mixed precision against
plain FP64 on the same matrix.

Workload (default "mixed-4m"): X = U diag(sigma) V^T, m = 4,000,000,
n = 256, sigma log-spaced 1 -> 1e-5, stored in FP32 (synthetic, seeded, drawn
on the GPU); Rademacher sketch with k = 768 rows, 2 passes (Algorithm 3).
One step = one rcholqr_factor call on X already resident in HBM.  The FP64
leg factors the same values promoted exactly to FP64.

Prints one JSON line.  `value` is the mixed-precision leg's GB/s of X
(m n 4 bytes / time per step).  `roofline` describes the slowest kernel phase
of that leg, timed live with HIP events recorded by the library on its
stream; `cpu_baseline` is the FP64 CPU oracle timed on a bounded sample of
rows of the same matrix on this host.
"""
import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm": 8.0e12, "f64": 78.6e12, "f32": 157.3e12, "f16": 2.5e15, "i8": 5.0e15,
        "bf16x3": 2.5e15 / 6}

# Size of the plain copy whose FETCH_SIZE / WRITE_SIZE readings turn the
# counters of the other kernels into HBM bytes (--copy-probe).
COPY_PROBE_BYTES = 1 << 30
CSRC = os.path.join(ROOT, "paper_2210_09953_amd", "csrc")
SHARED_HEADERS = ("common.h", "kernels.h", "theta.h")

# The kernel that does the work of each phase, by precision, and its source.
PHASE_KERNEL = {
    "mixed": {"sketch": "rcq::sketch_i8_kernel", "small_qr": "rcq::hh_panel_kernel",
              "solve1": "rcq::trsm_bf3_kernel", "gram": "rcq::gram_bf3_kernel",
              "cholesky": "rcq::chol_kernel", "solve2": "rcq::trmm_bf3_kernel"},
    "f32": {"sketch": "rcq::sketch_dense_kernel", "small_qr": "rcq::hh_panel_kernel",
            "solve1": "rcq::trsm_bf3_kernel", "gram": "rcq::gram_bf3_kernel",
            "cholesky": "rcq::chol_kernel", "solve2": "rcq::trmm_bf3_kernel"},
    "f64": {"sketch": "rcq::sketch_dense_kernel", "small_qr": "rcq::hh_panel_kernel",
            "solve1": "rcq::trsm_kernel<double", "gram": "rcq::gram_kernel<double",
            "cholesky": "rcq::chol_kernel", "solve2": "rcq::trmm_kernel<double"},
}
KERNEL_SOURCE = (("sketch_i8", "mixed.hip"), ("sketch_", "sketch.hip"), ("count_", "sketch.hip"),
                 ("hh_", "small.hip"),
                 ("chol_", "small.hip"), ("make_bf3", "small.hip"), ("trsm_", "tall.hip"),
                 ("trmm_", "tall.hip"), ("gram_", "tall.hip"), ("make_panels", "tall.hip"))


def source_hash(kernel):
    """sha256 of the source file that defines `kernel` and the shared headers."""
    short = kernel.split("rcq::")[-1]
    for prefix, fname in KERNEL_SOURCE:
        if short.startswith(prefix):
            h = hashlib.sha256()
            for f in (fname,) + SHARED_HEADERS:
                with open(os.path.join(CSRC, f), "rb") as fh:
                    h.update(fh.read())
            return h.hexdigest()[:16]
    return None


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.md")


def pmc_per_kernel(run_dir, counter):
    """{kernel: (dispatches, mean counter value)} from one rocprofv3 --pmc run."""
    import sqlite3
    tot, disp = {}, {}
    for db in glob.glob(os.path.join(run_dir, "**", "*.db"), recursive=True):
        cur = sqlite3.connect(db).cursor()
        for name, cn, val, d in cur.execute(
                "select kernel_name, counter_name, value, dispatch_id from counters_collection"):
            if cn != counter:
                continue
            short = re.sub(r"\(.*", "", name).replace("void ", "").strip()
            tot[short] = tot.get(short, 0.0) + val
            disp.setdefault(short, set()).add(d)
    return {k: (len(disp[k]), tot[k] / len(disp[k])) for k in tot}


def summarize_pmc(workload, fetch_dir, write_dir, command):
    """Write profiles/traffic_<workload>.md: HBM bytes per dispatch of every
    library kernel, FETCH_SIZE and WRITE_SIZE (KiB) each scaled by what the
    counter reads for the plain copy of COPY_PROBE_BYTES bytes."""
    f = pmc_per_kernel(fetch_dir, "FETCH_SIZE")
    w = pmc_per_kernel(write_dir, "WRITE_SIZE")
    copy = "rcq::hbm_copy_kernel"
    if copy not in f or copy not in w:
        raise SystemExit("copy probe kernel missing from the counter runs (--copy-probe)")
    ff = COPY_PROBE_BYTES / (f[copy][1] * 1024.0)
    wf = COPY_PROBE_BYTES / (w[copy][1] * 1024.0)
    rows, kern = [], {}
    for k in sorted(set(f) & set(w)):
        if not k.startswith("rcq::") or k == copy:
            continue
        b = f[k][1] * 1024.0 * ff + w[k][1] * 1024.0 * wf
        kern[k] = {"dispatches": f[k][0], "fetch_kib": round(f[k][1], 1),
                   "write_kib": round(w[k][1], 1), "hbm_bytes": round(b), "src": source_hash(k)}
        rows.append(f"| `{k}` | {f[k][0]} | {f[k][1]:.1f} | {w[k][1]:.1f} | {b / 1e9:.4f} |")
    rec = {"workload": workload, "copy_bytes": COPY_PROBE_BYTES,
           "copy_fetch_kib": f[copy][1], "copy_write_kib": w[copy][1],
           "fetch_factor": ff, "write_factor": wf, "kernels": kern}
    txt = [f"# HBM traffic per dispatch, workload {workload}", "",
           "Commands (repository root, one MI355X; one counter per run):", "",
           "    " + command.replace("COUNTER", "FETCH_SIZE").replace("DIR", fetch_dir),
           "    " + command.replace("COUNTER", "WRITE_SIZE").replace("DIR", write_dir),
           "    python3 bench.py --workload " + workload + f" --summarize-pmc {fetch_dir} {write_dir}",
           "",
           f"Copy reference: {COPY_PROBE_BYTES} bytes read and written by `rcq::hbm_copy_kernel`;",
           f"FETCH_SIZE read {f[copy][1]:.1f} KiB (factor {ff:.4f}), "
           f"WRITE_SIZE read {w[copy][1]:.1f} KiB (factor {wf:.4f}).",
           "HBM bytes = FETCH_SIZE x 1024 x fetch factor + WRITE_SIZE x 1024 x write factor.",
           "", "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM GB |",
           "|---|---:|---:|---:|---:|"] + rows + ["", "Record read by bench.py:", "",
                                                  "    " + json.dumps(rec), ""]
    with open(traffic_file(workload), "w") as fh:
        fh.write("\n".join(txt))
    print("\n".join(txt))


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none or the kernel's source changed since."""
    try:
        with open(traffic_file(workload)) as fh:
            line = [l for l in fh if l.strip().startswith("{")][-1]
        rec = json.loads(line)["kernels"]
    except (OSError, IndexError, ValueError, KeyError):
        return None
    # Several instances may match (e.g. whole-tile and ragged-tail kernels of
    # a solve): the dominant one moves the most bytes.
    found = [v["hbm_bytes"] for k, v in rec.items()
             if k.startswith(kernel) and v.get("src") == source_hash(k)]
    return max(found) if found else None

WORKLOADS = {
    # name: (m, n, k, kind, sigma_min, value precision, x dtype bytes)
    "mixed-4m": dict(m=4_000_000, n=256, k=768, kind="rademacher", sigma=1e-5,
                     precision="mixed"),
    "mixed-1m": dict(m=1_000_000, n=256, k=768, kind="rademacher", sigma=1e-5,
                     precision="mixed"),
    "f64-gauss-1m": dict(m=1_000_000, n=200, k=600, kind="gaussian", sigma=1e-12,
                         precision="f64"),
    "f64-count-1m": dict(m=1_000_000, n=200, k=600, kind="countsketch", sigma=1e-12,
                         precision="f64"),
    "f32-gauss-1m": dict(m=1_000_000, n=200, k=600, kind="gaussian", sigma=1e-6,
                         precision="f32"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def phase_model(phase, m, n, k, kind, prec):
    """Algorithmic work of one phase: (flops, HBM bytes, matrix-core dtype).

    FP32 data (f32, mixed) goes through the tall phases on bf16 matrix cores
    with three-way splits: six bf16 products per FP32-accurate product, so
    their compute peak is the bf16 peak / 6 ("bf16x3")."""
    s = 8 if prec == "f64" else 4
    mm = "f64" if prec == "f64" else "bf16x3"
    if phase == "sketch":
        if kind == "countsketch":
            return float(m * n), float(m * n * s), "hbm"
        return 2.0 * m * k * n, float(m * n * s), ("i8" if prec == "mixed" else "f64")
    if phase in ("solve1", "solve2"):
        return float(m) * n * n, 2.0 * m * n * s, mm
    if phase == "gram":
        return float(m) * n * (n + 1), float(m * n * s), mm
    return 0.0, 0.0, "f64"


def phase_kernel(phase, kind, prec):
    if phase == "sketch" and kind == "countsketch":
        return "rcq::count_accum_kernel"
    return PHASE_KERNEL[prec][phase]


def roofline(phase, ms_per_launch, m, n, k, kind, prec, traffic=None):
    flops, nbytes, unit = phase_model(phase, m, n, k, kind, prec)
    kname = phase_kernel(phase, kind, prec)
    t_mem = nbytes / PEAK["hbm"]
    t_cmp = flops / PEAK[unit] if unit != "hbm" else 0.0
    t = ms_per_launch * 1e-3
    if t_cmp > t_mem:
        a = flops / t / 1e12
        return {"bound": "mfma", "achieved": round(a, 3), "peak": PEAK[unit] / 1e12,
                "unit": "TFLOP/s", "frac": round(a * 1e12 / PEAK[unit], 4), "traffic": traffic,
                "kernel": kname, "phase": phase, "dtype": unit, "ms_per_launch": round(ms_per_launch, 4),
                "flops_per_launch": flops, "bytes_per_launch": nbytes}
    a = nbytes / t / 1e9
    return {"bound": "hbm", "achieved": round(a, 1), "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
            "frac": round(a * 1e9 / PEAK["hbm"], 4), "traffic": traffic, "kernel": kname,
            "phase": phase,
            "ms_per_launch": round(ms_per_launch, 4), "flops_per_launch": flops,
            "bytes_per_launch": nbytes}


def quality(torch, X, Q, R, nsample=200000):
    """||Q^T Q - I||_2 (FP64 accumulation on the GPU) and the max column-wise
    relative residual ||X_j - (QR)_j|| / ||X_j|| on a row sample."""
    Qd = Q.double()
    G = Qd.T @ Qd
    G -= torch.eye(G.shape[0], dtype=G.dtype, device=G.device)
    orth = float(torch.linalg.matrix_norm(G.cpu(), ord=2))
    m = X.shape[0]
    idx = torch.linspace(0, m - 1, min(nsample, m), device=X.device).long()
    Xs, Qs = X[idx].double(), Qd[idx]
    res = Xs - Qs @ R
    col = torch.linalg.vector_norm(res, dim=0) / torch.linalg.vector_norm(Xs, dim=0)
    return orth, float(col.max())


def time_leg(torch, rq, X, k, kind, prec_code, steps, warmup, seed=1):
    m, n = X.shape
    dt = torch.float64 if prec_code == rq.F64 else torch.float32
    Q = rq.empty_fortran(m, n, dt)
    R = rq.empty_fortran(n, n, torch.float64)
    ws = torch.empty(rq.workspace_bytes(m, n, k, kind, 2, prec_code), dtype=torch.uint8,
                     device="cuda")
    for _ in range(warmup):
        rq.factor(X, k, seed, kind, 2, prec_code, ws=ws, Q=Q, R=R)
    torch.cuda.synchronize()
    st = rq.status(ws)
    if st != 0:
        raise RuntimeError(f"status {st}: {rq.error_string(st)}")
    rq.profile_enable(True)
    rq.profile_read()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        rq.factor(X, k, seed, kind, 2, prec_code, ws=ws, Q=Q, R=R)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    calls, phases = rq.profile_read()
    rq.profile_enable(False)
    phases = {p: v / max(calls, 1) for p, v in phases.items()}
    return ms, phases, Q, R


def reduced_leg(torch, rq, X, k, l, kind, prec_code, steps, warmup, seed=1):
    """Reduced RCholeskyQR (Algorithm 5) on the same X: Z = L X R^{-1}.
    Returns ms per call and ||S^T S - I||_2 of the sketch's orthonormal
    factor (outside the timed region)."""
    m, n = X.shape
    ws = torch.empty(int(rq.lib().rcholqr_reduced_workspace_bytes(m, n, k, l, kind, prec_code)),
                     dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        rq.reduced(X, k, l, seed, kind, prec_code, ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        Z, R = rq.reduced(X, k, l, seed, kind, prec_code, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = rq.status(ws)
    _, _, ex = rq.reduced(X, k, l, seed, kind, prec_code, want_s=True, ws=ws)
    S = ex["S"]
    orth_s = float(torch.linalg.matrix_norm(S.T @ S - torch.eye(n, dtype=S.dtype, device=S.device), 2))
    return ms, orth_s, st


def col_leg(torch, rq, X, k, kind, prec_code, steps, warmup, nblocks=4, seed=1):
    """Column-oriented RCholeskyQR (Algorithm 4) of the same X in nblocks
    equal column blocks, one C-ABI call per block (X_b read from X).
    Returns ms per whole factorisation and cond(Q)."""
    m, n = X.shape
    w = n // nblocks
    cq = rq.ColumnQR(m, n, k, seed, kind, prec_code)
    # one workspace for the largest call (the last block)
    cq.ws = torch.empty(int(rq.lib().rcholqr_col_block_workspace_bytes(m, n - w, w, k, kind,
                                                                       prec_code)),
                        dtype=torch.uint8, device="cuda")

    def run():
        cq.j = 0
        for b in range(nblocks):
            cq.append(X[:, b * w:(b + 1) * w])
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    s = torch.linalg.svdvals(cq.Q.double().T @ cq.Q.double())
    return ms, float(torch.sqrt(s[0] / s[-1]))


def rr_leg(torch, rq, X, k, kind, prec_code, steps, warmup, tau, passes=1, seed=1):
    """Rank-revealing RCholeskyQR (Algorithm 7) on the same X.  Returns ms per
    call (the rank read after the timed region), the rank and cond(Q)."""
    m, n = X.shape
    ws = torch.empty(int(rq.lib().rcholqr_rr_workspace_bytes(m, n, k, kind, prec_code, passes)),
                     dtype=torch.uint8, device="cuda")
    Q = rq.empty_fortran(m, n, X.dtype)
    R = rq.empty_fortran(n, n, torch.float64)
    piv = torch.empty(n, dtype=torch.int32, device="cuda")
    rank = torch.empty(1, dtype=torch.int32, device="cuda")
    L = rq.lib()
    import ctypes

    def call():
        code = L.rcholqr_rr(ctypes.c_void_p(X.data_ptr()), m, n, max(X.stride(1), m), k, seed,
                            kind, prec_code, passes, float(tau), 1.5,
                            ctypes.c_void_p(Q.data_ptr()), m,
                            ctypes.c_void_p(R.data_ptr()), n, ctypes.c_void_p(piv.data_ptr()),
                            ctypes.c_void_p(rank.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                            ws.numel(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        if code != 0:
            raise RuntimeError(f"rcholqr_rr: {code}")
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    r = int(rank.item())
    G = Q[:, :r].double().T @ Q[:, :r].double()
    s = torch.linalg.svdvals(G)
    orth = float(torch.linalg.matrix_norm(G - torch.eye(r, dtype=G.dtype, device=G.device), 2))
    return ms, r, float(torch.sqrt(s[0] / s[-1])), orth


def batched_leg(torch, rq, synth, steps, warmup, count=512):
    """The persistent batched engine on the batched configuration; value =
    GB/s of X (sum m n 4 bytes per call); roofline = HBM with the 2-pass
    algorithmic traffic 5 sum(m n) 4 bytes (read X for the sketch, read X and
    write Q1 in the solve, read Q1 and write Q in the product; the Gram reads
    the chunk it just wrote, from cache)."""
    shapes = synth.batched_shapes(count, seed=0)
    Xs = [synth.make_x_torch(mm, nn, 1e-4, seed=1000 + i, dtype=torch.float32)
          for i, (mm, nn, _) in enumerate(shapes)]
    eng = rq.BatchedEngine(Xs, [kk for _, _, kk in shapes], [1 + i for i in range(count)],
                           passes=2)
    for _ in range(warmup):
        eng.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        eng.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = eng.status()
    worst = 0.0
    for i in range(0, count, 16):  # every 16th problem: ||Q^T Q - I||_2
        Q = eng.Qs[i].double()
        nn = Q.shape[1]
        worst = max(worst, torch.linalg.matrix_norm(
            Q.T @ Q - torch.eye(nn, device=Q.device, dtype=torch.float64), 2).item())
    # the same launch replayed from a HIP graph
    eng.capture()
    eng.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        eng.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / steps
    # for comparison: the same problems through rcholqr_factor_batched (one
    # single-problem launch sequence per problem over the stream pool)
    pool = rq.BatchedFactor(Xs, [kk for _, _, kk in shapes], [1 + i for i in range(count)],
                            kind=rq.RADEMACHER, passes=2, precision=rq.MIXED)
    for _ in range(max(1, warmup)):
        pool.run()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        pool.run()
    e1.record()
    torch.cuda.synchronize()
    ms_pool = e0.elapsed_time(e1) / steps
    del pool
    xbytes = sum(mm * nn for mm, nn, _ in shapes) * 4
    achieved = 5 * xbytes / (ms * 1e-3) / 1e9
    out = {"value": round(xbytes / (ms * 1e-3) / 1e9, 2), "unit": "GB/s",
           "ms_per_step": round(ms, 4), "ms_graph_replay": round(ms_graph, 4),
           "stream_pool_ms": round(ms_pool, 4), "problems": count, "x_bytes": xbytes,
           "chunk_rows": eng.chunk, "statuses_nonzero": sum(1 for v in st if v != 0),
           "worst_orth": worst,
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0,
                        "unit": "GB/s", "frac": round(achieved / 8000.0, 4),
                        "algorithmic_bytes": 5 * xbytes}}
    del eng, Xs
    torch.cuda.empty_cache()
    return out


def adjoint_leg(torch, rq, synth, steps, warmup, m=1_000_000, n=128):
    """The differentiation configuration: 2-pass forward (FP32 X, Gaussian
    sketch, k = 3n) and the adjoint dX from dQ ~ N(0, 1) (m x n) and an
    upper triangular dR ~ N(0, 1), the first-pass Q recomputed by the
    backward's own kernels.  value = GB/s of X (m n 4 bytes) per
    forward + backward."""
    k = 3 * n
    X = synth.make_x_torch(m, n, 1e-6, seed=2, dtype=torch.float32)
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    dQ = rq.fortran(torch.randn(n, m, dtype=torch.float32, device="cuda", generator=g).T)
    dR = torch.triu(torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g))
    ws_f = torch.empty(rq.workspace_bytes(m, n, k, rq.GAUSSIAN, 2, rq.F32), dtype=torch.uint8,
                       device="cuda")
    ws_b = torch.empty(int(rq.lib().rcholqr_backward_workspace_bytes(m, n, rq.F32)),
                       dtype=torch.uint8, device="cuda")
    fwd = lambda: rq.factor(X, k, 1, rq.GAUSSIAN, 2, rq.F32, ws=ws_f, want_factors=True)
    Q, R, ex = fwd()
    dX = rq.backward(X, ex["Rs"], ex["Rp"], dQ, dR, precision=rq.F32, ws=ws_b)
    for _ in range(warmup):
        Q, R, ex = fwd()
        dX = rq.backward(X, ex["Rs"], ex["Rp"], dQ, dR, precision=rq.F32, dX=dX, ws=ws_b)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_f = t_b = 0.0
    for _ in range(steps):
        e[0].record()
        Q, R, ex = fwd()
        e[1].record()
        dX = rq.backward(X, ex["Rs"], ex["Rp"], dQ, dR, precision=rq.F32, dX=dX, ws=ws_b)
        e[2].record()
        torch.cuda.synchronize()
        t_f += e[0].elapsed_time(e[1])
        t_b += e[1].elapsed_time(e[2])
    t_f, t_b = t_f / steps, t_b / steps
    finite = bool(torch.isfinite(dX).all().item())
    out = {"value": round(m * n * 4 / ((t_f + t_b) * 1e-3) / 1e9, 2), "unit": "GB/s",
           "ms_forward": round(t_f, 4), "ms_backward": round(t_b, 4), "m": m, "n": n, "k": k,
           "sketch": "gaussian", "precision": "f32", "dX_finite": finite}
    del X, dQ, dR, Q, R, ex, dX, ws_f, ws_b
    torch.cuda.empty_cache()
    return out


def host_cpu():
    """lscpu's model, sockets, cores per socket and threads per core of this
    host, and the CPUs this process may run on (affinity)."""
    info = {}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket":
                "cores_per_socket", "Thread(s) per core": "threads_per_core", "CPU(s)": "cpus"}
        for line in out.splitlines():
            if ":" not in line:
                continue
            k, v = (t.strip() for t in line.split(":", 1))
            if k in keys and keys[k] not in info:
                info[keys[k]] = int(v) if v.isdigit() else v
    except Exception as e:  # lscpu missing: report what Python knows
        info["lscpu_error"] = str(e)
    if "sockets" in info and "cores_per_socket" in info:
        info["physical_cores"] = info["sockets"] * info["cores_per_socket"]
    info["affinity_cpus"] = len(os.sched_getaffinity(0))
    return info


def cpu_baseline(Xs_np, k, kind_code, budget_s=15.0):
    """FP64 CPU oracle (test infrastructure) on the first rows of X.

    A warm-up call loads the library and starts its threads; a timed call on
    16384 rows then sets the row count that fills about `budget_s` seconds
    (all phases but the k x n QR and the n x n Cholesky scale with rows)."""
    import numpy as np
    import oracle
    threads = oracle.threads()
    m_all, n = Xs_np.shape
    oracle.rcholqr(np.asfortranarray(Xs_np[:max(2048, n)]), k, 1, kind_code, passes=2)
    m0 = min(m_all, 16384)
    t0 = time.perf_counter()
    oracle.rcholqr(np.asfortranarray(Xs_np[:m0]), k, 1, kind_code, passes=2)
    t_small = time.perf_counter() - t0
    m1 = int(min(m_all, max(m0, m0 * budget_s / max(t_small, 1e-3))))
    m1 = max(n, (m1 // 1024) * 1024) if m1 > 1024 else m1
    t0 = time.perf_counter()
    out = oracle.rcholqr(np.asfortranarray(Xs_np[:m1]), k, 1, kind_code, passes=2)
    t = time.perf_counter() - t0
    return m1, t, threads, out["status"]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mixed-4m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--no-reduced-leg", action="store_true",
                    help="skip the Reduced RCholeskyQR figure")
    ap.add_argument("--no-col-leg", action="store_true",
                    help="skip the column-oriented (four-block) factorisation of the same X")
    ap.add_argument("--no-srht-leg", action="store_true",
                    help="skip the SRHT-sketch factorisation of the same X")
    ap.add_argument("--no-rr-leg", action="store_true",
                    help="skip the rank-revealing RCholeskyQR figure")
    ap.add_argument("--no-batched-leg", action="store_true",
                    help="skip the 512-problem batched-engine figure")
    ap.add_argument("--no-1m-leg", action="store_true",
                    help="skip the mixed m = 1e6 figure (and its oracle comparison)")
    ap.add_argument("--no-adjoint-leg", action="store_true",
                    help="skip the forward + adjoint figure (m = 1e6, n = 128, FP32)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=45.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain copy of 1 GiB (byte-counter reference)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs into profiles/traffic_<workload>.md")
    ap.add_argument("--pmc-command", default="rocprofv3 --pmc COUNTER -d DIR -o run -- "
                    "python3 bench.py --steps 2 --warmup 1 --no-cpu --no-fp64-leg "
                    "--no-reduced-leg --no-srht-leg --no-col-leg --no-rr-leg --no-batched-leg "
                    "--no-1m-leg --no-adjoint-leg --copy-probe")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.workload, args.summarize_pmc[0], args.summarize_pmc[1],
                      args.pmc_command)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2210_09953_amd as rq
    import synth

    W = WORKLOADS[args.workload]
    m, n, k = W["m"], W["n"], W["k"]
    kind = {"gaussian": rq.GAUSSIAN, "rademacher": rq.RADEMACHER,
            "countsketch": rq.COUNTSKETCH}[W["kind"]]
    prec = W["precision"]
    prec_code = {"f64": rq.F64, "f32": rq.F32, "mixed": rq.MIXED}[prec]
    xdt = torch.float64 if prec == "f64" else torch.float32
    xbytes = 8 if prec == "f64" else 4

    log(f"[bench] generating X {m}x{n} sigma_min={W['sigma']} on cuda:0")
    X = synth.make_x_torch(m, n, W["sigma"], seed=0, dtype=xdt, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] value leg: precision={prec} kind={W['kind']} k={k} "
        f"steps={args.steps} warmup={args.warmup}")
    ms, phases, Q, R = time_leg(torch, rq, X, k, kind, prec_code, args.steps, args.warmup)
    orth, res = quality(torch, X, Q, R)
    value = m * n * xbytes / (ms * 1e-3) / 1e9
    log(f"[bench] {prec}: {ms:.3f} ms/step {value:.1f} GB/s orth={orth:.2e} resid={res:.2e} "
        f"phases={ {p: round(v, 4) for p, v in phases.items()} }")
    dom = max(phases, key=phases.get)
    traffic = measured_traffic(args.workload, phase_kernel(dom, W["kind"], prec))
    roof = roofline(dom, phases[dom], m, n, k, W["kind"], prec, traffic)
    # The same model for every tall phase (context for the dominant one).
    phase_roof = {}
    for ph in ("sketch", "solve1", "gram", "solve2"):
        r = roofline(ph, phases[ph], m, n, k, W["kind"], prec,
                     measured_traffic(args.workload, phase_kernel(ph, W["kind"], prec)))
        phase_roof[ph] = {key: r[key] for key in ("bound", "achieved", "unit", "frac", "traffic")}
    if args.copy_probe:
        # Known-size plain copy for scaling the byte counters (outside the timed region).
        src = torch.empty(COPY_PROBE_BYTES, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        rq.device_copy(src, dst)
        torch.cuda.synchronize()
        del src, dst
    R_value = R.clone()
    del Q

    # Reduced RCholeskyQR on the same X (one pass over X; l extractor rows).
    red = None
    if not args.no_reduced_leg and kind != rq.COUNTSKETCH:
        l = min(256, 1024 - k)
        ms_r, orth_s, st_r = reduced_leg(torch, rq, X, k, l, kind, prec_code, args.steps,
                                         args.warmup)
        red = {"value": round(m * n * xbytes / (ms_r * 1e-3) / 1e9, 2), "unit": "GB/s",
               "ms_per_step": round(ms_r, 4), "l": l, "orth_S": orth_s, "status": st_r}
        log(f"[bench] reduced (l={l}): {ms_r:.3f} ms/step {red['value']} GB/s "
            f"||S^T S - I|| = {orth_s:.2e}")

    # The same factorisation with the SRHT sketch (the ±1 kinds share the
    # int8 path).
    srht = None
    if not args.no_srht_leg and kind == rq.RADEMACHER:
        ms_s, ph_s, Q_s, R_s = time_leg(torch, rq, X, k, rq.SRHT, prec_code, args.steps,
                                        args.warmup)
        orth_s2, res_s2 = quality(torch, X, Q_s, R_s)
        srht = {"value": round(m * n * xbytes / (ms_s * 1e-3) / 1e9, 2), "unit": "GB/s",
                "ms_per_step": round(ms_s, 4), "orth": orth_s2, "resid": res_s2,
                "phases_ms": {p: round(v, 4) for p, v in ph_s.items()}}
        log(f"[bench] srht: {ms_s:.3f} ms/step {srht['value']} GB/s orth={orth_s2:.2e} "
            f"resid={res_s2:.2e} sketch={ph_s.get('sketch', 0.0):.3f} ms")
        del Q_s, R_s

    # Column-oriented RCholeskyQR of the same X in four blocks.
    col = None
    if not args.no_col_leg and n % 4 == 0:
        ms_c, cond_c = col_leg(torch, rq, X, k, kind, prec_code, args.steps, args.warmup)
        col = {"value": round(m * n * xbytes / (ms_c * 1e-3) / 1e9, 2), "unit": "GB/s",
               "ms_per_step": round(ms_c, 4), "blocks": 4, "cond_Q": cond_c}
        log(f"[bench] column-oriented (4 blocks): {ms_c:.3f} ms/step {col['value']} GB/s "
            f"cond(Q) {cond_c:.3f}")

    # Rank-revealing RCholeskyQR on the same X.
    rrf = None
    if not args.no_rr_leg:
        tau = 1e-10
        ms_rr, r_rr, cond_q, _ = rr_leg(torch, rq, X, k, kind, prec_code, args.steps, args.warmup,
                                        tau)
        rrf = {"value": round(m * n * xbytes / (ms_rr * 1e-3) / 1e9, 2), "unit": "GB/s",
               "ms_per_step": round(ms_rr, 4), "tau": tau, "rank": r_rr, "cond_Q": cond_q}
        log(f"[bench] rank-revealing: {ms_rr:.3f} ms/step {rrf['value']} GB/s rank {r_rr} "
            f"cond(Q) {cond_q:.3f}")
        ms2, r2, cond2, orth2 = rr_leg(torch, rq, X, k, kind, prec_code, args.steps, args.warmup,
                                       tau, passes=2)
        rrf["two_pass"] = {"value": round(m * n * xbytes / (ms2 * 1e-3) / 1e9, 2),
                           "unit": "GB/s", "ms_per_step": round(ms2, 4), "rank": r2,
                           "orth": orth2}
        log(f"[bench] rank-revealing, 2 passes: {ms2:.3f} ms/step {rrf['two_pass']['value']} "
            f"GB/s rank {r2} ||Q^T Q - I|| = {orth2:.2e}")
        # the same shape at rank 64 (X's first 64 columns times a seeded
        # Gaussian 64 x n): the tall steps touch only the kept columns
        g = torch.Generator(device="cuda")
        g.manual_seed(5)
        G = torch.randn(64, n, dtype=torch.float64, device="cuda", generator=g)
        Xl = rq.fortran((X[:, :64].double() @ G).to(X.dtype))
        del G
        ms_l, r_l, cond_l, _ = rr_leg(torch, rq, Xl, k, kind, prec_code, args.steps,
                                      args.warmup, 1e-5)
        del Xl
        rrf["rank_64"] = {"value": round(m * n * xbytes / (ms_l * 1e-3) / 1e9, 2),
                          "unit": "GB/s", "ms_per_step": round(ms_l, 4), "tau": 1e-5,
                          "rank": r_l, "cond_Q": cond_l}
        log(f"[bench] rank-revealing, X of rank 64: {ms_l:.3f} ms/step "
            f"{rrf['rank_64']['value']} GB/s rank {r_l} cond(Q) {cond_l:.3f}")

    fp64 = None
    if not args.no_fp64_leg and prec != "f64":
        X64 = X.double()
        X64 = rq.fortran(X64)
        ms64, ph64, Q64, R64 = time_leg(torch, rq, X64, k, kind, rq.F64, args.steps,
                                        args.warmup)
        orth64, res64 = quality(torch, X64, Q64, R64)
        dR = float(torch.linalg.matrix_norm(R_value - R64) / torch.linalg.matrix_norm(R64))
        fp64 = {"value": round(m * n * xbytes / (ms64 * 1e-3) / 1e9, 2),
                "unit": "GB/s", "ms_per_step": round(ms64, 4), "orth": orth64,
                "resid": res64, "rel_diff_R_vs_value_leg": dR,
                "phases_ms": {p: round(v, 4) for p, v in ph64.items()},
                "speedup_of_value_leg": round(ms64 / ms, 3)}
        log(f"[bench] f64: {ms64:.3f} ms/step orth={orth64:.2e} resid={res64:.2e} dR={dR:.2e}")
        del Q64, X64

    # The batched configuration on the persistent batched engine: 512
    # problems, m uniform in [2000, 200000], n in {16, 32, 64, 96, 128},
    # k = 3n, sigma 1 -> 1e-4, FP32, Rademacher, 2 passes, one launch each.
    batched = None
    if not args.no_batched_leg:
        batched = batched_leg(torch, rq, synth, args.steps, args.warmup)
        log(f"[bench] batched engine: {batched['ms_per_step']:.3f} ms/step "
            f"{batched['value']} GB/s, HBM frac {batched['roofline']['frac']}, "
            f"worst orth {batched['worst_orth']:.2e}")

    # The benchmark spec's size, m = 1e6 (n, k, kind as the value leg), where the
    # fixed-size small steps weigh more; its Q and R are compared with the
    # FP64 oracle in the CPU section below.
    leg1m = None
    X1np = Q1np = R1np = None
    if not args.no_1m_leg and prec == "mixed" and m > 1_000_000:
        m1m = 1_000_000
        X1 = synth.make_x_torch(m1m, n, W["sigma"], seed=1, dtype=xdt, device="cuda")
        ms1, ph1, Q1, R1 = time_leg(torch, rq, X1, k, kind, prec_code, args.steps, args.warmup)
        orth1, res1 = quality(torch, X1, Q1, R1)
        small = ph1.get("small_qr", 0.0) + ph1.get("cholesky", 0.0)
        leg1m = {"value": round(m1m * n * xbytes / (ms1 * 1e-3) / 1e9, 2), "unit": "GB/s",
                 "ms_per_step": round(ms1, 4), "m": m1m, "orth": orth1, "resid": res1,
                 "phases_ms": {p: round(v, 4) for p, v in ph1.items()},
                 "small_steps_share": round(small / ms1, 3)}
        log(f"[bench] mixed m=1e6: {ms1:.3f} ms/step {leg1m['value']} GB/s orth={orth1:.2e} "
            f"small steps {small:.3f} ms")
        if not args.no_cpu:
            X1np = np.asfortranarray(X1.double().cpu().numpy())
            Q1np = Q1.double().cpu().numpy()
            R1np = R1.cpu().numpy()
        del X1, Q1, R1

    adj = None
    if not args.no_adjoint_leg:
        adj = adjoint_leg(torch, rq, synth, args.steps, args.warmup)
        log(f"[bench] adjoint (1e6 x 128, FP32): forward {adj['ms_forward']:.3f} ms, "
            f"backward {adj['ms_backward']:.3f} ms, {adj['value']} GB/s")

    cpu = None
    if not args.no_cpu:
        ms_rows = min(m, 1 << 21)
        Xs = X[:ms_rows].double().cpu().numpy()
        Xs = np.asfortranarray(Xs)
        log(f"[bench] cpu baseline (FP64 oracle) on up to {ms_rows} rows")
        m1, t, threads, st = cpu_baseline(Xs, k, kind, args.cpu_budget)
        cpu = {"value": round(m1 * n * xbytes / t / 1e9, 4), "unit": "GB/s", "cores": threads,
               "kind": "oracle", "host": host_cpu(),
               "sample": f"first {m1} rows of X (n={n}, k={k}, {W['kind']}, 2 passes, FP64), "
                         f"{t:.1f} s, status {st}"}
        log(f"[bench] cpu: {cpu}")
        if X1np is not None:
            # the m = 1e6 leg against the FP64 oracle on the same FP32 values
            import oracle
            t0 = time.perf_counter()
            ref = oracle.rcholqr(X1np, k, 1, kind, passes=2)
            t_or = time.perf_counter() - t0
            dR = float(np.linalg.norm(R1np - ref["R"]) / np.linalg.norm(ref["R"]))
            dQ = float(np.linalg.norm(Q1np - ref["Q"]) / np.linalg.norm(ref["Q"]))
            leg1m["oracle"] = {"rel_dR": dR, "rel_dQ": dQ, "status": int(ref["status"]),
                               "seconds": round(t_or, 1)}
            log(f"[bench] m=1e6 vs oracle: |dR|/|R| {dR:.2e} |dQ|/|Q| {dQ:.2e} ({t_or:.1f} s)")
            del X1np, Q1np, R1np, ref

    out = {
        "metric": "GB/s of X factored + ||Q^T Q - I||: mixed vs FP64 RCholQR, 1 MI355X",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "mixed": "i8+bf16+f32+f64"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "k": k, "sketch": W["kind"],
                   "passes": 2, "sigma_min": W["sigma"], "x_dtype": str(xdt).split(".")[-1],
                   "precision": prec},
        "orth": orth, "resid": res,
        "phases_ms": {p: round(v, 4) for p, v in phases.items()},
        "roofline": roof,
        "phase_rooflines": phase_roof,
        "fp64": fp64,
        "reduced": red,
        "srht": srht,
        "column_oriented": col,
        "rank_revealing": rrf,
        "cpu_baseline": cpu,
        "batched": batched,
        "mixed_1m": leg1m,
        "adjoint": adj,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
