#!/usr/bin/env python3
"""Benchmark: sketched Krylov f(A)b solves per second on one MI355X.

Default workload (the largest single-GPU configuration): nonsymmetric 3D
upwind convection-diffusion, 7-point stencil on a 256^3 grid
(n = 16,777,216), Pe = 100, scaled to ||A||_inf = 1e3; exp(-1e-3 A) B for a
block B of 8 right-hand sides ~ N(0,1) (seeds 50..57), interleaved row by row;
Krylov dimension m = 200, truncation k = 4, SRHT sketch with s = 800 rows
(seed 5); FP32 basis (108 GB for the block) with FP64 accumulation, FP64
sketched QR / least squares / exp / combination.  One step = one complete
block solve (basis, sketch, least squares, f(H_hat) e_1 and combination for
all 8 right-hand sides) with B and the result resident in HBM; `value` counts
f(A)b results (right-hand sides) per second.

Prints one JSON line.  Besides the contract fields it carries
  roofline      the dominant kernel (the fused update + sketch pass): its
                algorithmic bytes per launch (the per-step byte count of the
                hot-path scope table: the update reads w~ and the window and
                writes the new vector) over its mean launch duration, timed
                with HIP events on the solve stream;
  cpu_baseline  the CPU oracle (full Arnoldi f_m, numpy/scipy FP64) timed on
                the host cores: one full solve where it takes seconds, else a
                bounded sample (stated in `sample`);
and in config: relative error of the timed result against the oracle (per
right-hand side), p50/p99 latency, algorithmic HBM GB/s of the whole solve,
and the FP64-basis rate of the same method (the plain FP64 GPU path).

--workload convdiff3d_128_exp: the same operator family at 128^3 (Pe = 50),
one right-hand side, m = 100, SRHT s = 400.
--workload lap3d_80_invsqrt times the sketched Gram-Schmidt basis
(Algorithm 3) on the paper's timing problem instead: A^{-1/2} b for the 3D
Laplacian with N = 80 (n = 512,000), m = 120, an SRHT sketch of
floor(1.05 m) = 126 rows, LSQR for the least squares.  By default the
Gram-Schmidt step on the sketch runs twice (--basis sketched_gs2): with so
few sketch rows one pass leaves Theta V far from orthonormal.  Its dominant
kernel is the update u_i = w - V_{i-1} r_i, its oracle Algorithm 3 with the
exact least-squares solution; it also reports the error against Arnoldi's f_m.
--workload rgg_2p20_invsqrt times the whitened basis (Section 2.1.2) on a
random geometric graph Laplacian with 2^20 nodes, (A + 1e-3 I)^{-1/2}, m = 150,
where the truncated basis alone loses its conditioning; --workload
convdiff2d_352_exp the variable-coefficient convection-diffusion of
Section 5.1.1 (CSR, exp).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "f(A)b solves/s at relerr≤1e-6 vs FP64 oracle; HBM GB/s; p50/p99 latency"
HBM_PEAK_GBPS = 8000.0


def algorithmic_bytes_bg(n, nrhs, m, esize, lsqr_iters):
    """Bytes per solve and per kernel class for the sketched Gram-Schmidt basis
    (stencil operator).  Step i (1..m): the apply pass reads u_{i-1}; the
    update reads u_0..u_{i-1} (the stencil source among them) and writes u_i.
    Start: read b, write u_0.  LSQR: per iteration one product with V_m and
    one with V_m^T (m vectors each) plus about 6 FP64 vectors of its own.
    Combine: read m vectors, write the FP64 result."""
    vec = n * nrhs * esize
    apply_ = m * vec
    update = sum(i + 1 for i in range(1, m + 1)) * vec
    start = n * nrhs * 8 + vec
    lsqr = lsqr_iters * (2 * m * vec + 6 * n * nrhs * 8)
    combine = m * vec + n * nrhs * 8
    return {"dots_per_launch": apply_ / m, "update_per_launch": update / m,
            "solve": apply_ + update + start + lsqr + combine}


def algorithmic_bytes_whitened(n, m, k, esize, nnz, wat, lsqr_iters):
    """Bytes per solve and per kernel class for the whitened basis on a CSR
    operator (one rhs): truncated steps 1..wat (the last one is discarded by
    the whitening), the in-place transform of wat vectors, Algorithm 1 steps
    wat..m; CSR arrays (8 B per nonzero + 4 B per row) and the FP64 product
    (written by the first pass of a step, read by the second) per step."""
    vec = n * esize
    csr = 8 * nnz + 4 * (n + 1)
    wb = 8 * n
    wat = wat if wat > 0 else m + 1
    nt_steps = range(1, min(wat, m) + 1)
    bg_steps = range(wat, m + 1) if wat <= m else range(0)
    dots = sum(min(i, k) * vec + csr + wb for i in nt_steps) + sum(vec + csr + wb for i in bg_steps)
    update = sum(min(i, k) * vec + wb + vec for i in nt_steps) + sum(i * vec + wb + vec for i in bg_steps)
    nupd = len(nt_steps) + len(bg_steps)
    whiten = 2 * wat * vec if wat <= m else 0
    start = 8 * n + vec
    lsqr = lsqr_iters * (2 * m * vec + 48 * n)
    combine = m * vec + 8 * n
    return {"dots_per_launch": dots / max(1, nupd), "update_per_launch": update / max(1, nupd),
            "solve": dots + update + whiten + start + lsqr + combine}


def algorithmic_bytes(n, nrhs, m, k, esize, nnz=None):
    """Bytes the method must move per solve and per kernel class.

    The scope-table count (the hot path's two passes per step as separate
    kernels): step i (1..m) reads the window of min(i, k) vectors and writes
    w~ (first pass), then reads w~ and the window and writes u_i (second
    pass), i.e. (2 min(i,k) + 3) vectors per step; a CSR operator adds its
    arrays (8 B per nonzero + 4 B per row) per step; the combination reads m
    vectors; b in and the result out are 16 B per row and rhs.

    The fused count is what the two fused kernels here must move at least:
    the first pass reads the window (its newest member is the matvec source)
    and writes nothing long; the second reads the window again and writes
    u_i (w~ is recomputed from the window, never stored); a CSR operator's
    FP64 product is written by the product kernel and read by both passes.
    """
    vec = n * nrhs * esize
    win = sum(min(i, k) for i in range(1, m + 1))
    mat = 0 if nnz is None else 8 * nnz + 4 * (n + 1)
    # scope-table count
    dots = win * vec + m * vec + m * mat
    update = (win + 2 * m) * vec
    solve = dots + update + m * vec + 16 * n * nrhs
    # fused count
    fdots = win * vec
    fupdate = (win + m) * vec
    if nnz is not None:
        wb = 8 * n * nrhs
        fdots += m * (mat + wb)
        fupdate += m * wb
    fsolve = fdots + fupdate + (n * nrhs * 8 + vec) + m * vec + n * nrhs * 8
    return {"dots_per_launch": dots / m, "update_per_launch": update / m, "solve": solve,
            "fused_dots_per_launch": fdots / m, "fused_update_per_launch": fupdate / m, "fused_solve": fsolve}


# Per workload: the basis it is timed with, its dominant kernel (the name
# rocprofv3 reports for the FP32 variant), the counter summary of that kernel
# and the sources that define it (a summary counts only while they are unchanged).
CSRC = "paper_2212_12758_amd/csrc/"
BENCH = {
    "convdiff3d_256_exp_8rhs": {
        "basis": "truncated",
        "kernel": "k_update (Gram-Schmidt update + norm + fused SRHT), 8 rhs",
        "pmc_kernel": "k_update<float, 0, 1, false, 11, 8, 4>",
        "traffic_file": os.path.join(ROOT, "profiles", "traffic_k_update_convdiff3d_256_exp_8rhs.json"),
        "sources": [CSRC + "k_basis.h", CSRC + "k_basis_part.inc", CSRC + "fab_dev.h"],
        "operator": "3D upwind convection-diffusion 7-point 256^3, Pe=100", "f": "exp(-1e-3 A)",
    },
    "convdiff3d_128_exp": {
        "basis": "truncated",
        "kernel": "k_update (Gram-Schmidt update + norm + fused SRHT)",
        "pmc_kernel": "k_update<float, 0, 1, false, 11, 1, 4>",
        "traffic_file": os.path.join(ROOT, "profiles", "traffic_k_update_convdiff3d_128_exp.json"),
        "sources": [CSRC + "k_basis.h", CSRC + "k_basis_part.inc", CSRC + "fab_dev.h"],
        "operator": "3D upwind convection-diffusion 7-point 128^3, Pe=50", "f": "exp(-1e-3 A)",
    },
    "convdiff2d_352_exp": {
        "basis": "truncated",
        "kernel": "k_update (Gram-Schmidt update + norm + fused SRHT), CSR operator",
        "pmc_kernel": "k_update<float, 1, 1, false, 9, 1, 2>",
        "traffic_file": os.path.join(ROOT, "profiles", "traffic_k_update_convdiff2d_352_exp.json"),
        "sources": [CSRC + "k_basis.h", CSRC + "k_basis_part.inc", CSRC + "fab_dev.h"],
        "operator": "2D variable-coefficient convection-diffusion 352^2 (Section 5.1.1), CSR", "f": "exp(-t A)",
    },
    "rgg_2p20_invsqrt": {
        "basis": "whitened",
        "kernel": "update passes (k_update of the truncated steps, then k_bg_update after whitening), CSR",
        "pmc_kernel": "k_update<float, 1, 1, false, 11, 1, 2>",
        "traffic_file": os.path.join(ROOT, "profiles", "traffic_k_update_rgg_2p20_invsqrt.json"),
        "sources": [CSRC + "k_basis.h", CSRC + "k_basis_part.inc", CSRC + "fab_dev.h"],
        "operator": "random geometric graph Laplacian, 2^20 nodes, mean degree ~10, CSR", "f": "(A + 1e-3 I)^{-1/2}",
    },
    "lap3d_80_invsqrt": {
        "basis": "sketched_gs2",
        "kernel": "k_bg_update (u_i = w - V_{i-1} r_i over all previous vectors)",
        "pmc_kernel": "k_bg_update<float, 0, true>",
        "traffic_file": os.path.join(ROOT, "profiles", "traffic_k_bg_update_lap3d_80_invsqrt.json"),
        "sources": [CSRC + "k_bg.hip", CSRC + "k_basis.h", CSRC + "fab_dev.h"],
        "operator": "3D Laplacian 7-point 80^3 (T_N = tridiag(-1, 2, -1))", "f": "A^{-1/2}",
    },
}
CALIBRATION_BYTES = 4 << 28   # the 1 GiB copy of --calibrate-copy


def kernel_source_hash(workload="convdiff3d_256_exp_8rhs"):
    import hashlib

    h = hashlib.sha256()
    for f in BENCH[workload]["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload="convdiff3d_256_exp_8rhs"):
    """HBM bytes per launch of the workload's dominant kernel from the committed
    counter summary, or None when its sources changed since the counters were taken."""
    try:
        with open(BENCH[workload]["traffic_file"]) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    return t["bytes_per_launch"] if t.get("source_sha256") == kernel_source_hash(workload) else None


def _pmc_rows(d, counter):
    import csv
    import glob

    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection*.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def summarize_pmc(fetch_dir, write_dir, workload="convdiff3d_256_exp_8rhs"):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the workload's dominant
    kernel, each scaled by the same counter on a copy kernel of known size (the
    1 GiB copy of --calibrate-copy), written to the traffic summary read by
    measured_traffic()."""
    cfg = BENCH[workload]
    out = {"kernel": cfg["pmc_kernel"], "workload": workload, "source_sha256": kernel_source_hash(workload)}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _pmc_rows(d, counter)
        copies = [v for k, v in rows if "copyBuffer" in k]
        upd = [v for k, v in rows if cfg["pmc_kernel"] in k]
        if not copies or not upd:
            raise SystemExit(f"{counter}: no calibration copy or {cfg['pmc_kernel']} dispatches in {d}")
        cal = max(copies)
        factor = CALIBRATION_BYTES / (cal * 1024.0)
        out[key] = {"counter": counter, "calibration_copy_kib": cal, "factor": factor,
                    "kernel_mean_kib": sum(upd) / len(upd), "dispatches": len(upd),
                    "bytes_per_launch": factor * 1024.0 * sum(upd) / len(upd)}
    out["bytes_per_launch"] = out["fetch"]["bytes_per_launch"] + out["write"]["bytes_per_launch"]
    with open(cfg["traffic_file"], "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def arena_bytes(w, nrhs):
    """Workspace for one FP64-basis solve of the workload (the FP32 attempt's
    FP64 fallback must fit too): the basis, the LSQR vector, an FP64 product
    buffer, plus 1 GiB for partials and the dense tail."""
    n, m = w.n, w.m
    nel = n * nrhs
    ldv = (nel + 63) // 64 * 64
    return max(6 << 30, (m + 1) * ldv * 8 + 2 * nel * 8 + (1 << 30))


def oracle_sample_fm(Aor, b, f, m, m_sample=20):
    """CPU oracle time for one full-Arnoldi f_m at dimension m.  When a full
    run would take minutes, a bounded sample: the oracle as it stands at
    m_sample < m steps, scaled linearly by m / m_sample.  Every Arnoldi step
    costs at least as much as any earlier one (one product with A, then
    Gram-Schmidt against all previous vectors), so the scaled time is a lower
    bound on the full solve's time and the rate an upper bound."""
    from oracle import krylov

    ms = min(m, m_sample)
    t0 = time.perf_counter()
    krylov.fm(Aor, b, f, ms)
    t = time.perf_counter() - t0
    if ms == m:
        return t, f"one full solve (m={m}, {t:.1f} s)"
    return t * m / ms, (f"bounded sample: the oracle's f_m at m={ms} on right-hand side 0 took {t:.1f} s, scaled "
                        f"by {m}/{ms} (a lower bound on the full solve's time: later steps cost more)")


def serving_main(args):
    """The serving mix: Poisson arrivals of single-rhs requests of mixed n, m
    and f (workloads.serving_mix), served by the context's request loop
    (continuous batching; queued requests on a shared resident matrix with
    the same parameters merged into block solves), FP32 basis with the
    automatic precision and least-squares policies at tol = 1e-6, SRHT
    sketch (as in the paper's experiments; --sketch sparse_sign).

    1. closed loop: every request queued at once; the makespan gives the
       saturated throughput;
    2. open loop: the trace replayed at 0.8 x that rate (exponential gaps
       from the workload's seed): value = requests / (last completion - first
       arrival), p50/p99 of submit-to-completion latency;
    3. the plain FP64 path: the same requests, FP64 basis, one blocking solve
       at a time (its throughput is 1 / mean service time; its latencies are
       those of a single server fed the same trace);
    4. accuracy: the oracle's f_m for a sample of requests (both paths).

    The context's serving streams (12) run concurrently only on as many
    hardware queues: HIP's default of 4 per process would serialise them, so
    this mode asks for 16 (GPU_MAX_HW_QUEUES, read when HIP starts;
    --hw-queues, at most 32)."""
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    import numpy as np
    import torch

    import workloads as W
    from paper_2212_12758_amd import Context, make_params

    nreq = args.requests
    reqs, gaps = W.serving_mix(nreq=nreq)
    nev = len(gaps)
    print(f"serving mix: {nreq} requests, {nev} arrival events", file=sys.stderr, flush=True)
    ctx = Context(0, arena_bytes=args.arena_gb << 30)
    pool = {}
    mats = []
    for r in reqs:
        if r.pool >= 0:
            if r.pool not in pool:
                pool[r.pool] = ctx.matrix(r.op)
            mats.append(pool[r.pool])
        else:
            mats.append(ctx.matrix(r.op))
    # right-hand sides: N(0,1) from a per-request seeded device generator
    bs, outs = [], []
    for r in reqs:
        g = torch.Generator(device="cuda")
        g.manual_seed(1_000_000 + r.rid)
        bs.append(torch.randn(r.op.n, generator=g, dtype=torch.float64, device="cuda"))
        outs.append(torch.empty_like(bs[-1]))
    torch.cuda.synchronize()

    def params(r, prec, tol):
        return make_params(r.m, r.k, r.s, args.sketch, 8, r.sketch_seed, prec, "auto", tol)

    p32 = [params(r, "auto", 1e-6) for r in reqs]

    def run(arrivals):
        """Submit request i at arrivals[event of i] (seconds from start);
        returns (makespan from first arrival, latencies in ms, infos)."""
        handles = [None] * nreq
        t0 = time.perf_counter()
        i = 0
        while i < nreq:
            due = arrivals[reqs[i].event]
            now = time.perf_counter() - t0
            if due > now:
                time.sleep(min(due - now, 0.002))
                continue
            handles[i] = ctx.submit(mats[i], bs[i], reqs[i].f, p32[i], outs[i])
            i += 1
        infos = [h.wait()[0] for h in handles]
        t_end = time.perf_counter() - t0
        lat = np.array([inf["latency_us"] for inf in infos]) / 1e3
        return t_end, lat, infos

    # warm-up: a few requests of each kind (graph-free served path; builds caches)
    for i in range(min(16, nreq)):
        ctx.submit(mats[i], bs[i], reqs[i].f, p32[i], outs[i]).wait()
    torch.cuda.synchronize()
    # 1. closed loop
    t_sat, lat_sat, _ = run(np.zeros(nev))
    rate_sat = nreq / t_sat
    print(f"closed loop: {t_sat:.2f} s, {rate_sat:.1f} solves/s", file=sys.stderr, flush=True)
    # 2. open loop at 0.8 x the saturated rate
    lam = 0.8 * rate_sat * nev / nreq           # arrival events per second
    arrivals = np.concatenate([[0.0], np.cumsum(gaps[:-1])]) / lam
    t_open, lat, infos = run(arrivals)
    value = nreq / t_open
    res32 = [o.clone() for o in outs]
    blocks = np.array([inf["block_rhs"] for inf in infos])
    print(f"open loop: {t_open:.2f} s, {value:.1f} solves/s, p50 {np.percentile(lat, 50):.2f} ms "
          f"p99 {np.percentile(lat, 99):.2f} ms", file=sys.stderr, flush=True)
    # 3. plain FP64 path, one request at a time
    p64 = [params(r, "fp64", 1e-6) for r in reqs]
    serv = np.zeros(nreq)
    infos64 = []
    for i in range(nreq):
        ts = time.perf_counter()
        _, inf64 = ctx.solve(mats[i], bs[i], reqs[i].f, p64[i], outs[i])
        torch.cuda.synchronize()
        serv[i] = time.perf_counter() - ts
        infos64.append(inf64[0])
    rate64 = nreq / serv.sum()
    done, lat64 = 0.0, np.zeros(nreq)
    for i in range(nreq):
        a = arrivals[reqs[i].event]
        done = max(done, a) + serv[i]
        lat64[i] = (done - a) * 1e3
    print(f"plain fp64: {rate64:.1f} solves/s", file=sys.stderr, flush=True)
    res64 = [o.clone() for o in outs]
    # every served result against the plain FP64 path's (on the GPU)
    e_vs64 = np.array([float(torch.linalg.norm(res32[i] - res64[i]) / torch.linalg.norm(res64[i]))
                       for i in range(nreq)])
    # 4. accuracy on a sample (the smallest requests, every f kind and both
    # kinds of matrix), oracle timed as the CPU baseline
    from oracle import krylov, operators

    order = sorted(range(nreq), key=lambda i: reqs[i].op.n)
    sample = order[:args.oracle_sample]
    c0 = time.perf_counter()
    errs32, errs64 = [], []
    for i in sample:
        r = reqs[i]
        b = bs[i].cpu().numpy()
        ref = krylov.fm(operators.as_matrix(r.op), b, r.f, r.m)
        errs32.append(krylov.relerr(res32[i].cpu().numpy(), ref))
        errs64.append(krylov.relerr(res64[i].cpu().numpy(), ref))
    tcpu = time.perf_counter() - c0
    for A in set(mats):
        A.destroy()
    ctx.close()
    errs32, errs64 = np.array(errs32), np.array(errs64)
    basis_bytes = sum(r.op.n * (r.m + 1) * 4 for r in reqs)
    line = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": nreq, "warmup": 16,
        "ms_per_step": 1e3 * t_open / nreq, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": "serving_mix", "requests": nreq, "arrival_events": nev,
            "operators": "2D 5-point / 3D 7-point Dirichlet Laplacians, n log-uniform in [2^14, 2^21]",
            "f": "exp(-tA) (||tA|| log-uniform [1, 50]), A^{1/2}, (A + 1e-3 I)^{-1/2}",
            "m": "U[30, 200]", "k": "U{2, 3, 4}", "s": "2m", "sketch": args.sketch,
            "shared_matrix_fraction": float(np.mean([r.pool >= 0 for r in reqs])),
            "arena_GB": args.arena_gb, "basis_GB_total": basis_bytes / 1e9,
            "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
            "saturated_solves_per_s": rate_sat, "arrival_rate_solves_per_s": 0.8 * rate_sat,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "closed_loop_p50_ms": float(np.percentile(lat_sat, 50)),
            "block_rhs_histogram": {str(int(g)): int((blocks == g).sum()) for g in np.unique(blocks)},
            "fell_back": int(sum(inf["fell_back"] for inf in infos)),
            "refined": int(sum(inf["ls_iters"] > 0 for inf in infos)),
            "plain_fp64_solves_per_s": rate64, "fp32_over_plain_fp64": value / rate64,
            "saturated_over_plain_fp64": rate_sat / rate64,
            "relerr_vs_plain_fp64_all_max": float(e_vs64.max()),
            "relerr_vs_plain_fp64_all_median": float(np.median(e_vs64)),
            "plain_fp64_p50_ms": float(np.percentile(lat64, 50)), "plain_fp64_p99_ms": float(np.percentile(lat64, 99)),
            "oracle_sample": len(sample), "relerr_vs_oracle_max": float(errs32.max()),
            "relerr_vs_oracle_median": float(np.median(errs32)),
            "meets_tol_fraction": float(np.mean(errs32 <= 1e-6)),
            "plain_fp64_relerr_vs_oracle_max": float(errs64.max()),
        },
        "roofline": None,
        "cpu_baseline": {"value": len(sample) / tcpu, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
                         "sample": f"f_m by full Arnoldi (FP64, numpy/scipy) for the {len(sample)} smallest requests "
                                   f"of the mix (n <= {reqs[sample[-1]].op.n}), {tcpu:.1f} s"},
    }
    if args.dump_requests:
        # per-request record of both paths (for studying where the time goes)
        recs = [{"n": r.op.n, "m": r.m, "k": r.k, "f": r.f.kind + (f" {r.f.p}" if r.f.kind == "pow" else ""),
                 "pool": r.pool,
                 "block_rhs": int(infos[i]["block_rhs"]), "latency_ms": float(lat[i]),
                 "fell_back": int(infos[i]["fell_back"]), "ls_iters": int(infos[i]["ls_iters"]),
                 "err_est": float(infos[i]["err_est"]), "fp64_service_ms": 1e3 * float(serv[i]),
                 "fp64_ls_iters": int(infos64[i]["ls_iters"])} for i, r in enumerate(reqs)]
        with open(args.dump_requests, "w") as fh:
            json.dump(recs, fh)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed solves (default: 10 for the 8-rhs "
                                                             "workload, 20 otherwise)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing (profiling runs)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-basis comparison run")
    ap.add_argument("--prec", default="auto", choices=["auto", "fp32", "fp64"],
                    help="basis precision policy (auto: FP32 + estimates + FP64 fallback)")
    ap.add_argument("--ls", default="auto", choices=["auto", "sketch", "none", "lsqr", "gram"],
                    help="least-squares policy (auto: sketch-and-solve + gate + LSQR refinement)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU: turn two rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE outputs into the traffic summary")
    ap.add_argument("--basis", default=None, choices=["truncated", "sketched_gs", "sketched_gs2", "whitened"],
                    help="basis construction (default: the workload's)")
    ap.add_argument("--requests", type=int, default=4096, help="serving_mix: number of requests")
    ap.add_argument("--arena-gb", type=int, default=16, help="serving_mix: arena budget (admission binds)")
    ap.add_argument("--oracle-sample", type=int, default=24, help="serving_mix: requests checked by the oracle")
    ap.add_argument("--hw-queues", type=int, default=16, help="serving_mix: GPU_MAX_HW_QUEUES for this process")
    ap.add_argument("--dump-requests", default=None,
                    help="serving_mix: write a JSON list of per-request records (both paths) to this file")
    ap.add_argument("--sketch", default="srht", choices=["srht", "sparse_sign"], help="serving_mix: sketch")
    ap.add_argument("--workload", default="convdiff3d_256_exp_8rhs", choices=sorted(BENCH) + ["serving_mix"],
                    help="convdiff3d_256_exp_8rhs (default: 256^3, 8 rhs), convdiff3d_128_exp, "
                         "lap3d_80_invsqrt (Algorithm 3), rgg_2p20_invsqrt (whitened), convdiff2d_352_exp")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, workload=args.workload)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the solve is not sharded "
                                   "across GPUs; N > 1 is not supported", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "serving_mix":
        serving_main(args)
        return

    import numpy as np
    import torch

    import workloads as W
    from paper_2212_12758_amd import Context, make_params

    cfg = BENCH[args.workload]
    basis = args.basis or cfg["basis"]
    bg = basis in ("sketched_gs", "sketched_gs2")
    whitened = basis == "whitened"
    w = W.config(args.workload)
    n, nrhs = w.n, w.nrhs
    steps = args.steps if args.steps is not None else (10 if nrhs > 1 else 20)
    print(f"bench {args.workload}: n={n} nrhs={nrhs} m={w.m} k={w.k} s={w.s} {w.sketch}", file=sys.stderr,
          flush=True)
    b = W.rhs(n, w.b_seed, nrhs) if w.b_seed >= 0 else None
    if b is None:   # the sin(pi x) sin(pi y) start vector of the 2D workload
        b = W.sine_rhs(int(round(n ** 0.5)))
    ctx = Context(0, arena_bytes=arena_bytes(w, nrhs))
    A = ctx.matrix(w.op)
    bd = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    out = torch.empty_like(bd)
    p32 = make_params(w.m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, args.prec, args.ls, 1e-6, basis=basis)
    p64 = make_params(w.m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, "fp64", args.ls, 1e-10, basis=basis)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    info = None
    for _ in range(args.warmup):
        _, info = ctx.solve(A, bd, w.f, p32, out)
    # timed region: K complete solves (replayed HIP graphs of the launch sequence)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        _, info = ctx.solve(A, bd, w.f, p32, out)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = steps * nrhs / elapsed
    print(f"timed {steps} solves: {1e3 * elapsed / steps:.2f} ms per solve", file=sys.stderr, flush=True)
    res32 = out.cpu().numpy()
    esize = 8 if info[0]["prec_used"] == 2 else 4
    nnz = None if hasattr(w.op, "coeff") else len(w.op[1])
    ab32 = algorithmic_bytes(n, nrhs, w.m, w.k, esize, nnz)
    if bg:
        ab32.update(algorithmic_bytes_bg(n, nrhs, w.m, esize, info[0]["ls_iters"]))
    elif whitened:
        ab32.update(algorithmic_bytes_whitened(n, w.m, w.k, esize, nnz, info[0]["whitened_at"],
                                               info[0]["ls_iters"]))
    if bg or whitened:   # these passes have no separate scope-table count
        for key in ("dots_per_launch", "update_per_launch", "solve"):
            ab32["fused_" + key] = ab32[key]

    # kernel timing region: the same K solves with direct launches and a HIP
    # event pair around every launch of the dominant kernel on its stream
    ctx.profile([ctx.K_UPDATE, ctx.K_DOTS])
    for c in range(5):
        ctx.profile_read(c, reset=True)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for _ in range(steps):
        ctx.solve(A, bd, w.f, p32, out)
    torch.cuda.synchronize()
    prof_elapsed = time.perf_counter() - p0
    nlaunch, tot_ms = ctx.profile_read(ctx.K_UPDATE, reset=True)
    nd, dots_ms = ctx.profile_read(ctx.K_DOTS, reset=True)
    ctx.profile([])
    upd_ms = tot_ms / max(1, nlaunch)
    achieved = ab32["update_per_launch"] / (upd_ms * 1e-3) / 1e9 if upd_ms > 0 else None
    dots_us = 1e3 * dots_ms / max(1, nd)
    print(f"profiled: k_update {1e3 * upd_ms:.1f} us, k_dots {dots_us:.1f} us per launch", file=sys.stderr,
          flush=True)

    fp64_rate = None
    res64 = None
    if not args.no_fp64:
        out64 = torch.empty_like(bd)
        ctx.solve(A, bd, w.f, p64, out64)
        torch.cuda.synchronize()
        k64 = max(2, steps // 4)
        s0 = time.perf_counter()
        for _ in range(k64):
            ctx.solve(A, bd, w.f, p64, out64)
        torch.cuda.synchronize()
        fp64_rate = k64 * nrhs / (time.perf_counter() - s0)
        res64 = out64.cpu().numpy()
        del out64
        print(f"fp64 basis: {fp64_rate:.2f} solves/s", file=sys.stderr, flush=True)
    A.destroy()
    ctx.close()
    del ctx, bd, out
    torch.cuda.empty_cache()

    cpu = None
    relerr = None
    relerr_rhs = None
    relerr64 = None
    relerr_fm = None
    oracle_what = None
    if not args.no_cpu_baseline:
        from oracle import closed_form, krylov, operators
        from oracle import sketch as osk

        Aor = operators.as_matrix(w.op)
        b0 = np.ascontiguousarray(b if nrhs == 1 else b[:, 0])
        if nrhs > 1:
            # the converged exp(-tA) B (Kronecker-sum closed form) equals f_m at
            # m = 200 here (||tA|| = 1); the oracle's full Arnoldi is timed on a sample
            ref = closed_form.kronecker_exp_fAb(w.op, w.f.alpha, b)
            oracle_what = "exp(-tA) B by the Kronecker-sum closed form (equal to f_m at this m)"
            tcpu, sample = oracle_sample_fm(Aor, b0, w.f, w.m)
            cpu = {"value": 1.0 / tcpu, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
                   "sample": f"f_m by full Arnoldi (FP64, numpy/scipy) for one right-hand side of the same "
                             f"workload (n={n}, m={w.m}): {sample}; at least {tcpu:.0f} s per solve"}
        else:
            c0 = time.perf_counter()
            if bg:
                sk = osk.Sketch(w.sketch, n, w.s, w.sketch_seed, w.zeta)
                ref = krylov.sgs(Aor, b, w.f, w.m, sk, passes=2 if basis == "sketched_gs2" else 1)["f"]
                what = (f"Algorithm 3 with the exact least squares (FP64, numpy/scipy, "
                        f"{'two' if basis == 'sketched_gs2' else 'one'} Gram-Schmidt pass(es) on the sketch)")
            elif whitened:
                sk = osk.Sketch(w.sketch, n, w.s, w.sketch_seed, w.zeta)
                ref = krylov.whitened(Aor, b, w.f, w.m, w.k, sk)["f"]
                what = "the truncated basis whitened and continued by Algorithm 1, exact least squares (FP64)"
            else:
                ref = krylov.fm(Aor, b, w.f, w.m)
                what = "f_m by full Arnoldi (FP64, numpy/scipy)"
            tcpu = time.perf_counter() - c0
            oracle_what = what
            cpu = {"value": 1.0 / tcpu, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
                   "sample": f"one full solve of the same workload: {what} at n={n}, m={w.m}, {tcpu:.1f} s"}
            if bg or whitened:
                relerr_fm = krylov.relerr(res32, krylov.fm(Aor, b, w.f, w.m))
        R = ref.reshape(n, nrhs)
        relerr_rhs = [krylov.relerr(res32.reshape(n, nrhs)[:, q], R[:, q]) for q in range(nrhs)]
        relerr = max(relerr_rhs)
        if res64 is not None:
            relerr64 = max(krylov.relerr(res64.reshape(n, nrhs)[:, q], R[:, q]) for q in range(nrhs))

    lat_ms = np.array(lat) * 1e3
    line = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if esize == 4 else "f64", "data": "synthetic",
        "config": {
            "workload": args.workload, "operator": cfg["operator"],
            "n": n, "nrhs": nrhs, "f": cfg["f"], "m": w.m, "k": None if bg else w.k, "s": w.s, "sketch": w.sketch,
            "basis": basis, "storage": "fp32" if esize == 4 else "fp64",
            "accumulate": "fp64", "value_counts": "f(A)b results (right-hand sides) per second",
            "block_solves_per_s": steps / elapsed,
            "relerr_vs_oracle": relerr, "relerr_vs_oracle_per_rhs": relerr_rhs, "oracle": oracle_what,
            "meets_tol": (relerr is not None and relerr <= 1e-6) or None,
            "m_used": info[0]["m_used"], "prec_policy": args.prec, "ls_policy": args.ls,
            "prec_used": {1: "fp32", 2: "fp64"}.get(info[0]["prec_used"]), "fell_back": info[0]["fell_back"],
            "ls_iters": info[0]["ls_iters"], "err_est": max(i["err_est"] for i in info),
            "ls_gate": max(i["ls_gate"] for i in info), "round_est": max(i["round_est"] for i in info),
            "conv_est": max(i["conv_est"] for i in info),
            "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
            "hbm_algorithmic_GBps": ab32["solve"] * (steps / elapsed) / 1e9,
            "hbm_algorithmic_GBps_fused_count": ab32["fused_solve"] * (steps / elapsed) / 1e9,
            "fp64_basis_solves_per_s": fp64_rate, "fp64_relerr_vs_oracle": relerr64,
            "fp32_over_fp64": (value / fp64_rate) if fp64_rate else None,
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBPS) if achieved else None,
                     "traffic": measured_traffic(args.workload),
                     "kernel": cfg["kernel"],
                     "bytes_per_launch": ab32["update_per_launch"],
                     "bytes_per_launch_fused_count": ab32["fused_update_per_launch"],
                     "mean_launch_us": upd_ms * 1e3,
                     "launches": nlaunch, "timing": "HIP events around each launch, direct launches, "
                     f"{steps} solves ({1e3 * prof_elapsed / steps:.2f} ms/solve in that region)",
                     "dots_kernel_mean_us": dots_us,
                     "dots_kernel_GBps": ab32["dots_per_launch"] / (dots_us * 1e-6) / 1e9 if dots_us > 0 else None},
        "cpu_baseline": cpu,
    }
    if bg or whitened:
        line["config"]["relerr_vs_arnoldi_fm"] = relerr_fm
    if whitened:
        line["config"]["whitened_at"] = info[0]["whitened_at"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
