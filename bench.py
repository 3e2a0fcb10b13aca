#!/usr/bin/env python3
"""Benchmark: matrix-free subspace-Hamiltonian SpMV on one MI355X.

A step is one matrix-free SpMV ``y = H_S x`` over the whole subspace (diagonal, group scan,
ladder-integer ranges, hash probes, projector refinement, accumulation), with the subspace,
hash table, operator tables and vectors resident in HBM.  The default workload is the largest
single-GPU configuration: a random 16-orbital molecular Hamiltonian (h ~ N(0, 0.1), (pq|rs) ~
N(0, 0.01) with 8-fold symmetry, Jordan-Wigner ladder terms) on the Cartesian product of 1500
alpha and 1500 beta strings of weight 5 (2.25M determinants), in FP64.

Output: one JSON line.  ``value`` = stored matrix elements (structural nonzeros of H_S)
processed per second of SpMV.  ``roofline`` prices the SpMV kernel's algorithmic bytes
against the 8 TB/s HBM peak.  ``cpu_baseline`` times the CPU oracle (term-by-term, binary
search) on the host cores on a row sample of the same input, lowest of 5 runs at all host
threads and at one thread.  Extra keys report the ground-state solve time (GPU Lanczos, FP64),
the work counters, and the same SpMV measurement on the 6x6 XXZ workload (one vector) and the
200-qubit heavy-hex workload (8 vectors, the block-Lanczos SpMM).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matrix elements/s in matrix-free SpMV; ground-state solve s; serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
# the SpMV kernel, the row engine it runs and its launch
KERNEL_SOURCES = ["paper_2603_18731_amd/csrc/engine.h", "paper_2603_18731_amd/csrc/matvec.h",
                  "paper_2603_18731_amd/csrc/device.h", "paper_2603_18731_amd/csrc/spmv_impl.h"]


def kernel_digest():
    """Digest of the SpMV kernel's sources (ties a stored counter profile to the code)."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions/s: 256 CUs x 4 SIMDs, 4 cycles each


def stored_traffic(workload, dtype, nvec, capacity, key="hbm_bytes_per_launch"):
    """HBM bytes per SpMV launch (or, with key="valu_insts_per_launch", VALU wave instructions)
    from the committed counter profile of this workload, or None when there is none, it was
    taken on other kernel sources or with another hash-table size.  The profile records
    FETCH_SIZE and WRITE_SIZE per dispatch (KiB) and the factors that scale them to the bytes a
    plain copy of known size moves."""
    path = os.path.join(ROOT, "profiles", "k_matvec_%s_%s_nvec%d.md" % (workload, dtype, nvec))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("traffic:"):
                for kv in line.split()[1:]:
                    k, v = kv.split("=")
                    vals[k] = v
    if vals.get("source_digest") != kernel_digest() or int(vals.get("capacity", -1)) != capacity:
        return None
    return float(vals[key]) if key in vals else None


def calibrate_copy():
    """A plain device copy of known size, profiled to scale FETCH_SIZE / WRITE_SIZE."""
    import torch

    n = 64 << 20  # doubles: 512 MiB
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 3}))


def algorithmic_bytes(N, W, probes, hits, nvec, esz):
    """Bytes the method must move per SpMV: per row the key (8W), the diagonal (8), x_i and
    y_i (2 * esz * nvec); per probe one 8-byte slot; per hit the key compare (8W) and the
    gathered x_j (esz * nvec)."""
    return N * (8 * W + 8 + 2 * esz * nvec) + probes * 8 + hits * (8 * W + esz * nvec)


def cpu_model():
    """The host CPU's model name (lscpu), or the platform string."""
    import platform
    import subprocess

    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return platform.processor() or platform.machine()


def gather_ceiling():
    """Random-gather rate of the device for buffers of 256 KiB .. 1 GiB (the bench-only
    microbenchmark library, not part of the C-ABI)."""
    import ctypes

    import torch

    path = os.path.join(ROOT, "paper_2603_18731_amd", "libqsd_bench.so")
    lib = ctypes.CDLL(path)
    lib.qsdbench_gather_rate.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    lib.qsdbench_gather_rate.restype = ctypes.c_int
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for kib in (256, 1024, 2048, 4096, 8192, 32768, 131072, 524288, 1048576):
        for ilp in (1, 2, 4, 8):
            r = ctypes.c_double()
            rc = lib.qsdbench_gather_rate(kib << 10, ilp, ctypes.byref(r), stream)
            if rc != 0:
                raise SystemExit("gather benchmark failed (%d)" % rc)
            print(json.dumps({"buffer_kib": kib, "ilp": ilp, "loads_per_s": r.value}), flush=True)


def make_workload(name):
    import workloads as wl

    if name == "xxz6x6":
        w = wl.c2_xxz6x6()
    elif name == "tfim12":
        w = wl.c1_tfim12()
    elif name == "fermi16":
        w = wl.c3_molecular()
    elif name == "fermi16_300":
        w = wl.c3_molecular(300, 300)
    elif name == "heavyhex200":
        w = wl.c4_heavy_hex()
    else:
        raise SystemExit("unknown workload %s" % name)
    return w


def cpu_baseline(w, nnz_total, budget_s=20.0):
    """Times the CPU oracle's SpMV (plain C, OpenMP over rows, term by term with binary search)
    on a random row sample sized to the budget, lowest of 5 runs (the paper's convention), at
    all host threads and at one thread; the rate is the sample's share of the stored elements
    per second."""
    import numpy as np

    from oracle import rowwise as orw
    from oracle import subspace as osub

    ck = osub.canonical_keys(w.keys)
    N = ck.shape[0]
    rng = np.random.default_rng(0)
    x = rng.normal(size=N)
    threads = orw.max_threads()
    # cost per row at all threads, from a small probe
    rows = np.sort(rng.choice(N, size=min(N, 512), replace=False))
    t0 = time.perf_counter()
    orw.matvec_c(ck, w.ops, x, rows)
    per_row = (time.perf_counter() - t0) / len(rows)
    out = {}
    # 5 runs at all threads take ~half the budget, 5 at one thread the other half
    for label, nthr, share in (("all", threads, 0.5), ("one", 1, 0.5)):
        per_row_t = per_row * (threads / nthr if nthr < threads else 1.0)
        nrow = int(max(64, min(N, budget_s * share / 5 / max(per_row_t, 1e-9))))
        rs = np.sort(rng.choice(N, size=nrow, replace=False))
        best = float("inf")
        for _ in range(5):
            t0 = time.perf_counter()
            orw.matvec_c(ck, w.ops, x, rs, nthreads=nthr)
            best = min(best, time.perf_counter() - t0)
        out[label] = (nrow, best)
    nrow, t = out["all"]
    nrow1, t1 = out["one"]
    return {"value": nnz_total * (nrow / N) / t, "unit": "matrix elements/s", "cores": threads, "kind": "oracle",
            "sample": "%d random rows of %d at %d threads (lowest of 5); rate = the rows' share of the %d stored "
                      "elements per second" % (nrow, N, threads, nnz_total),
            "value_1thread": nnz_total * (nrow1 / N) / t1,
            "sample_1thread": "%d random rows, 1 thread, lowest of 5" % nrow1,
            "cpu_model": cpu_model(), "matvec_s": t * N / nrow, "matvec_s_1thread": t1 * N / nrow1}


def serve_bench(args):
    """Serving workload: requests drawn from the three families (TFIM-12, XXZ 6x6 at weight 18,
    16-orbital molecular), subspace sizes log-uniform in [1e3, smax], each a ground-state solve to
    1e-10 (FP64 SpMV) or 1e-7 (FP32 SpMV).  Baseline: the plain FP64 single-vector solver serving
    the same requests FIFO one at a time; its per-request solve times are measured, and its
    latencies under the same arrival times follow from the FIFO recurrence."""
    import numpy as np
    import torch

    import paper_2603_18731_amd as qsd
    import workloads as wl
    from paper_2603_18731_amd import serve

    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    specs = wl.serving_requests(args.serve_requests, smax=args.serve_smax)
    h, eri = wl.molecular_integrals(16, 3)
    fam_ops = {"tfim12": wl.tfim_chain(12, 1.0, 1.0, True), "xxz6x6": wl.xxz_grid_6x6(),
               "fermi16": wl.molecular_terms(h, eri)}
    ops = {k: qsd.operator_from_termlist(v) for k, v in fam_ops.items()}
    hams = []
    nnzs = []
    csr_min = (1 << 15) if args.serve_csr else None
    for i, (fam, size, sub_seed) in enumerate(specs):
        keys = wl.serving_subspace(fam, size, sub_seed)
        H = qsd.SubspaceHamiltonian(qsd.Subspace(keys, fam_ops[fam].n_qubits), ops[fam])
        hams.append(H)
        # stored-matrix size, for the CSR memory budget (a pass over the rows at setup)
        nnzs.append(H.N + H.work_counts()[1] if csr_min is not None and H.N >= csr_min else 0)
        if (i + 1) % 32 == 0:
            print("# built %d/%d request operators (%.0f s)" % (i + 1, len(specs), time.perf_counter() - t_setup),
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    sizes = np.array([H.N for H in hams])
    n = len(hams)
    print("# %d requests, %d rows in total, setup %.0f s" % (n, sizes.sum(), time.perf_counter() - t_setup),
          file=sys.stderr, flush=True)
    tol = 1e-10 if args.dtype == "f64" else 1e-7
    max_iter = 300

    # FIFO baselines, one request at a time: the plain FP64 single-vector matrix-free Lanczos, and
    # (with stored-CSR serving) the same solver on the CSR matrix, built inside the request's
    # service time, for every request the server would serve from CSR
    def fifo_solve(i, use_csr):
        H = hams[i]
        if use_csr and csr_min is not None and H.N >= csr_min:
            A = qsd.CsrMatrix(H, qsd.INDEX_I32, lower_mirror=True)
            r = A.lanczos(tol=1e-10, max_iter=max_iter, v0="uniform", raise_on_nonconv=False)
            del A
            return r
        return H.lanczos(tol=1e-10, max_iter=max_iter, v0="uniform", raise_on_nonconv=False)

    def fifo_service(use_csr, label):
        service = np.zeros(n)
        e_fifo = np.zeros(n)
        iters = np.zeros(n, dtype=np.int64)
        for i in range(n):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, _, info = fifo_solve(i, use_csr)
            torch.cuda.synchronize()
            service[i] = time.perf_counter() - t0
            e_fifo[i], iters[i] = e, info["iterations"]
            if (i + 1) % 64 == 0:
                print("# fifo %s %d/%d solved (%.1f s of service so far)" % (label, i + 1, n, service.sum()),
                      file=sys.stderr, flush=True)
        return service, e_fifo, iters

    service, e_fifo, iters_fifo = fifo_service(False, "matrix-free")
    mu_fifo = n / service.sum()
    service_csr = None
    if csr_min is not None:
        service_csr, e_fifo_csr, _ = fifo_service(True, "csr")

    free, _ = torch.cuda.mem_get_info()
    budget = int(0.85 * free)

    def run(arrivals, label):
        srv = serve.Server(budget, max_iter=max_iter, spmv_dtype=args.dtype, csr_min_rows=csr_min)
        reqs = [serve.Request(i, hams[i], arrival=float(arrivals[i]), tol=tol, nnz=nnzs[i]) for i in range(n)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = srv.run(reqs, progress=lambda k: k % 32 == 0 and print(
            "# %s: %d/%d done (%.1f s)" % (label, k, n, time.perf_counter() - t0), file=sys.stderr, flush=True))
        span = max(r.finished for r in done)
        lat = np.array([r.latency for r in sorted(done, key=lambda r: r.rid)])
        en = np.array([r.energy for r in sorted(done, key=lambda r: r.rid)])
        err = np.abs(en - e_fifo) / np.abs(e_fifo)
        res = dict(serve.percentiles(lat), solves_per_s=n / span, makespan_s=span,
                   converged=int(sum(r.status == 2 for r in done)),
                   energy_max_rel_err_vs_fp64=float(err.max()), peak_hbm_gb=srv.peak_used / 1e9,
                   peak_active=srv.peak_active, csr_requests=int(sum(r.used_csr for r in done)))
        print("# %s: %s" % (label, json.dumps(res)), file=sys.stderr, flush=True)
        return res

    closed = run(np.zeros(n), "closed loop")
    mu = closed["solves_per_s"]
    fifo_closed_lat = serve.fifo_latencies(np.zeros(n), service)
    out_open = {}
    fifo_open = {}
    fifo_csr = None
    if service_csr is not None:
        fifo_csr = {"solves_per_s": n / service_csr.sum(), "service_s_total": float(service_csr.sum()),
                    "closed_loop": serve.percentiles(serve.fifo_latencies(np.zeros(n), service_csr)),
                    "energy_max_rel_diff_vs_matrix_free": float(np.max(np.abs(e_fifo_csr - e_fifo) / np.abs(e_fifo)))}
    arrivals = {}
    for f in (0.7, 0.9):
        arr = serve.poisson_arrivals(n, f * mu, seed=5 + int(f * 10))
        arrivals[f] = arr
        out_open["lambda_%.1f_mu" % f] = dict(run(arr, "open loop %.1f mu" % f), rate_per_s=f * mu)
        fifo_open["lambda_%.1f_mu" % f] = serve.percentiles(serve.fifo_latencies(arr, service))
        if fifo_csr is not None:
            fifo_csr["lambda_%.1f_mu" % f] = serve.percentiles(serve.fifo_latencies(arr, service_csr))
    # one FIFO open-loop pass run for real (the like-for-like baseline: from stored CSR when the
    # server uses it), beside the latencies its measured service times predict
    real_csr = fifo_csr is not None
    arr = arrivals[0.9]
    print("# real FIFO pass (%s) at 0.9 mu arrivals" % ("csr" if real_csr else "matrix-free"), file=sys.stderr,
          flush=True)
    lat_real = serve.fifo_run(arr, lambda i: (fifo_solve(i, real_csr), torch.cuda.synchronize()))
    fifo_real = {"baseline": "csr" if real_csr else "matrix_free", "arrivals": "lambda_0.9_mu",
                 **serve.percentiles(lat_real),
                 "predicted": serve.percentiles(serve.fifo_latencies(arr, service_csr if real_csr else service))}
    print("# real FIFO pass: %s" % json.dumps(fifo_real), file=sys.stderr, flush=True)
    out = {
        "metric": "serve p50/p99 ms; solves/s",
        "value": mu,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": 0,
        "ms_per_step": closed["makespan_s"] * 1e3 / n,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "serve_%d_requests_1e3_%.0e%s" % (n, args.serve_smax, "_csr" if csr_min else ""),
                   "rows_total": int(sizes.sum()), "csr_min_rows": csr_min,
                   "tol": tol, "max_iter": max_iter, "hbm_budget_gb": budget / 1e9},
        "serve": {"closed_loop": closed, **out_open},
        "fifo_fp64_single_vector": {"solves_per_s": mu_fifo, "service_s_total": float(service.sum()),
                                    "closed_loop": serve.percentiles(fifo_closed_lat), **fifo_open,
                                    "iterations_mean": float(iters_fifo.mean())},
        "fifo_run_for_real": fifo_real,
    }
    if fifo_csr is not None:
        out["fifo_fp64_single_vector_csr"] = fifo_csr
    print(json.dumps(out), flush=True)


def precision_compare(args):
    """FP64 vs FP32 SpMV (FP32 elements and vectors, FP64 row accumulation) on one workload: the
    SpMV time of each (autotuned separately), and the ground-state energy of single-vector and
    block-8 Lanczos with either SpMV (orthogonalization, the tridiagonal solve and the residual
    test stay FP64), with the FP32 energy's relative difference from the FP64 one."""
    import numpy as np
    import torch

    import paper_2603_18731_amd as qsd

    torch.cuda.set_device(0)
    w = make_workload(args.workload)
    sub = qsd.Subspace(w.keys, w.ops.n_qubits)
    H = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(w.ops))
    st = torch.cuda.current_stream()
    out = {"workload": w.name, "N": sub.N}
    for dt, name in ((torch.float64, "f64"), (torch.float32, "f32")):
        tune = H.autotune(nvec=1, dtype=dt, reps=2)
        x = torch.rand(sub.N, dtype=dt, device="cuda")
        y = torch.empty_like(x)
        H.matvec(x, out=y)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
        for a, b in ev:
            a.record(st)
            H.matvec(x, out=y)
            b.record(st)
        torch.cuda.synchronize()
        out["spmv_ms_" + name] = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        out["autotune_" + name] = tune
        for block in (1, 8):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, _, info = H.lanczos(tol=1e-10 if name == "f64" else 1e-7, max_iter=300 if block == 1 else 80,
                                   v0="uniform", spmv_dtype=name, block=block, raise_on_nonconv=False)
            key = "%s_b%d" % (name, block)
            out["energy_" + key] = e
            out["solve_s_" + key] = time.perf_counter() - t0
            out["iterations_" + key] = info["iterations"]
            out["converged_" + key] = bool(info["converged"])
            print("# %s: %s SpMV %.3f ms, block %d: %.12f in %.3f s (%d steps)" % (
                w.name, name, out["spmv_ms_" + name], block, e, out["solve_s_" + key], info["iterations"]),
                file=sys.stderr, flush=True)
    # the oracle's ground energy of this workload, where one was computed (tests/golden, written by
    # a script that runs only the CPU oracle)
    with open(os.path.join(ROOT, "tests", "golden", "energies.json")) as f:
        golden = json.load(f)
    e_or = golden.get(w.name, {}).get("energy")
    out["energy_oracle"] = e_or
    for block in (1, 8):
        e64 = out["energy_f64_b%d" % block]
        out["energy_rel_err_f32_b%d" % block] = abs(out["energy_f32_b%d" % block] - e64) / abs(e64)
        for name in ("f64", "f32"):
            if e_or is not None:
                out["energy_rel_err_vs_oracle_%s_b%d" % (name, block)] = abs(out["energy_%s_b%d" % (name, block)] - e_or) / abs(e_or)
    print(json.dumps({"precision_compare": out}), flush=True)


def csr_compare(args):
    """Matrix-free vs stored-CSR solve on one workload: CSR build time (two-pass and
    lower-triangle), device memory, SpMV time of both operators, Lanczos time and energy."""
    import numpy as np
    import torch

    import paper_2603_18731_amd as qsd

    torch.cuda.set_device(0)
    w = make_workload(args.workload)
    sub = qsd.Subspace(w.keys, w.ops.n_qubits, max_load=args.max_load)
    op = qsd.operator_from_termlist(w.ops)
    H = qsd.SubspaceHamiltonian(sub, op)
    tune = None
    if args.schedule == "auto":
        tune = H.autotune(reps=2, load=args.max_load == 0.0)
    else:
        H.schedule = int(args.schedule)
    N = sub.N
    print("# %s: N=%d, autotuned %s" % (w.name, N, json.dumps(tune)), file=sys.stderr, flush=True)
    st = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(st)
            fn()
            b.record(st)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    x = torch.rand(N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    mf_ms = timed(lambda: H.matvec(x, out=y), 5)
    out = {"workload": w.name, "N": N, "matrix_free_spmv_ms": mf_ms}
    for lower in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A = qsd.CsrMatrix(H, qsd.INDEX_I32 if N < 2**31 else qsd.INDEX_I64, lower_mirror=lower)
        torch.cuda.synchronize()
        key = "lower_mirror" if lower else "two_pass"
        out["csr_build_s_" + key] = time.perf_counter() - t0
        print("# CSR build (%s): %.3f s, nnz %d, %.2f GB" % (key, out["csr_build_s_" + key], A.nnz, A.bytes / 1e9),
              file=sys.stderr, flush=True)
        if not lower:
            del A
    y2 = torch.empty_like(x)
    csr_ms = timed(lambda: A.matvec(x, out=y2), 10)
    out.update({"nnz": A.nnz, "csr_bytes": A.bytes, "csr_spmv_ms": csr_ms,
                "csr_spmv_gbs": (A.bytes + 3 * 8 * N) / (csr_ms / 1e3) / 1e9,
                "spmv_max_rel_diff": float(((y2 - y).abs().max() / y.abs().max()).item())})
    print("# SpMV: matrix-free %.3f ms, CSR %.3f ms (%.0f GB/s streamed)" % (mf_ms, csr_ms, out["csr_spmv_gbs"]),
          file=sys.stderr, flush=True)
    for mode, obj in (() if args.no_solve else (("csr", A), ("matrix_free", H))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, _, info = obj.lanczos(tol=1e-10, max_iter=300, v0="uniform", raise_on_nonconv=False)
        out["solve_s_" + mode] = time.perf_counter() - t0
        out["energy_" + mode] = e
        out["iterations_" + mode] = info["iterations"]
        print("# Lanczos (%s): %.12f in %.3f s, %d iterations" % (mode, e, out["solve_s_" + mode],
                                                                  info["iterations"]), file=sys.stderr, flush=True)
    if not args.no_solve:
        out["energy_rel_diff"] = abs(out["energy_csr"] - out["energy_matrix_free"]) / abs(out["energy_matrix_free"])
    print(json.dumps({"csr_vs_matrix_free": out}), flush=True)


def ramps_bench(args):
    """RAMPS on the full sampled subspace of --workload (Supplement, Algorithm S1, restricted to
    it): S_0 = the 64 strings of lowest diagonal energy, E = the ground energy of H restricted
    to S_0; then the ground energy on the trimmed subspace against the full one."""
    import numpy as np
    import torch

    import paper_2603_18731_amd as qsd

    torch.cuda.set_device(0)
    w = make_workload(args.workload)
    sub = qsd.Subspace(w.keys, w.ops.n_qubits)
    op = qsd.operator_from_termlist(w.ops)
    H = qsd.SubspaceHamiltonian(sub, op)
    d = H.diagonal()
    s0 = torch.argsort(d, stable=True)[:64].cpu().numpy()
    m0 = torch.zeros(sub.N, dtype=torch.uint8, device="cuda")
    m0[torch.from_numpy(s0).cuda()] = 1
    H0 = qsd.SubspaceHamiltonian(sub.select(m0), op)
    E, _, _ = H0.lanczos(tol=1e-12, max_iter=64)
    A = qsd.CsrMatrix(H, lower_mirror=True)
    e_full, _, info_full = A.lanczos(tol=1e-10, max_iter=300, raise_on_nonconv=False)
    del A
    out = {"workload": w.name, "N_full": sub.N, "S0": int(len(s0)), "E": E, "energy_full": e_full, "runs": []}
    print("# S_0: 64 lowest-diagonal strings, E = %.10f; full-subspace energy %.10f" % (E, e_full), file=sys.stderr,
          flush=True)
    for tau in (1e-3, 1e-4, 1e-5, 1e-6):
        try:
            H.ramps(s0, E, tau, max_depth=args.ramps_depth, max_frontier=1 << 26)  # warm-up
        except qsd.QsdError as exc:
            out["runs"].append({"tau": tau, "error": str(exc)})
            print("# RAMPS tau %.0e: %s" % (tau, exc), file=sys.stderr, flush=True)
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mask, info = H.ramps(s0, E, tau, max_depth=args.ramps_depth, max_frontier=1 << 26)
        torch.cuda.synchronize()
        t_ramps = time.perf_counter() - t0
        small = sub.select(mask)
        Hs = qsd.SubspaceHamiltonian(small, op)
        t0 = time.perf_counter()
        e_small, _, _ = Hs.lanczos(tol=1e-10, max_iter=300, raise_on_nonconv=False)
        t_solve = time.perf_counter() - t0
        r = {"tau": tau, "ramps_s": t_ramps, "solve_trimmed_s": t_solve, "energy_trimmed": e_small,
             "energy_rel_diff": abs(e_small - e_full) / abs(e_full), **info}
        out["runs"].append(r)
        print("# RAMPS tau %.0e: %d of %d strings, %d paths, %d levels, %.3f s; energy %.10f (full %.10f)" % (
            tau, info["selected"], sub.N, info["paths"], info["levels"], t_ramps, e_small, e_full), file=sys.stderr,
            flush=True)
    print(json.dumps({"ramps": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fermi16", help="fermi16 (1500 x 1500), fermi16_300 (300 x 300), "
                    "xxz6x6, heavyhex200 or tfim12")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--nvec", type=int, default=1)
    ap.add_argument("--max-load", type=float, default=0.0, help="hash load factor (0 = library default)")
    ap.add_argument("--schedule", default="auto", help="SpMV schedule bits, or 'auto' for the autotuner")
    ap.add_argument("--split", type=int, default=-1, help="hash split qubit (0 = none; -1 = the autotuner "
                    "decides, or none with a fixed schedule)")
    ap.add_argument("--group-order", default="default", choices=["default", "weight", "mask", "parts"],
                    help="group order: weight then flip mask, flip mask, halves flipped (alpha / beta) then "
                    "mask; default = parts for fermionic operators, weight for qubit operators")
    ap.add_argument("--no-extra", action="store_true", help="skip the XXZ and heavy-hex extra measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--gather-ceiling", action="store_true", help="measure the random-gather rate for "
                    "buffer sizes 256 KiB .. 1 GiB and exit")
    ap.add_argument("--calibrate-copy", action="store_true", help="run the plain-copy kernel used to scale "
                    "rocprofv3 FETCH_SIZE / WRITE_SIZE and exit")
    ap.add_argument("--ramps", action="store_true", help="RAMPS on --workload's subspace from its lowest "
                    "diagonal string; trimmed vs full ground energy")
    ap.add_argument("--ramps-depth", type=int, default=16)
    ap.add_argument("--csr-compare", action="store_true", help="matrix-free vs stored-CSR solve on --workload")
    ap.add_argument("--precision", action="store_true", help="FP64 vs FP32 SpMV and solves on --workload")
    ap.add_argument("--serve", action="store_true", help="serving benchmark: batched Lanczos requests with "
                    "Poisson arrivals against the FIFO single-vector solver")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-smax", type=float, default=2e6)
    ap.add_argument("--serve-csr", action="store_true", help="serve requests of >= 2^15 rows from stored CSR "
                    "matrices built at admission")
    args = ap.parse_args()
    if args.ramps:
        if args.gpus != 1:
            print("bench.py measures one GPU only (requested --gpus %d)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        ramps_bench(args)
        return
    if args.precision:
        precision_compare(args)
        return
    if args.csr_compare:
        if args.gpus != 1:
            print("bench.py measures one GPU only (requested --gpus %d)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        csr_compare(args)
        return
    if args.serve:
        if args.gpus != 1:
            print("bench.py measures one GPU only (requested --gpus %d)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        serve_bench(args)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gather_ceiling:
        gather_ceiling()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library does not shard the subspace SpMV across "
              "GPUs (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = make_workload(args.workload)
    r = measure_spmv(w, args.nvec, args.dtype, args.steps, args.warmup, args.max_load, args.schedule,
                     split=args.split, solve=not args.no_solve, group_order=args.group_order)
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "matrix elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": r["config"],
        "roofline": r["roofline"],
        "roofline_issue": r["roofline_issue"],
        "work": r["work"],
    }
    if "ground_state" in r:
        out["ground_state"] = r["ground_state"]
    if not args.no_extra and args.workload == "fermi16":
        # the other two large configurations, measured the same way (outside the headline)
        for name, nvec in (("xxz6x6", 1), ("heavyhex200", 8)):
            we = make_workload(name)
            re_ = measure_spmv(we, nvec, args.dtype, max(5, args.steps), args.warmup, 0.0, "auto", split=-1,
                               solve=False)
            out["extra_%s_nvec%d" % (we.name, nvec)] = {
                "value": re_["value"], "unit": "matrix elements/s", "ms_per_step": re_["ms_per_step"],
                "config": re_["config"], "roofline": re_["roofline"], "work": re_["work"]}
            del we
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, r["config"]["nnz"] * args.nvec)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "value_1thread",
                                                   "sample_1thread", "cpu_model")}
        print("# cpu oracle %.3f s per SpMV on %d threads, %.3f s on one (%s)" % (
            cb["matvec_s"], cb["cores"], cb["matvec_s_1thread"], cb["cpu_model"]), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def measure_spmv(w, nvec, dtype_name, steps, warmup, max_load, schedule, split=0, solve=True, group_order="default"):
    """Builds workload ``w`` on the device, counts its work, tunes (``schedule`` = "auto") and
    times ``steps`` SpMVs after ``warmup`` with HIP events on the launch stream."""
    import ctypes

    import numpy as np
    import torch

    import paper_2603_18731_amd as qsd

    t_setup = time.perf_counter()
    print("# workload %s: %d strings, %d qubits" % (w.name, w.keys.shape[0], w.ops.n_qubits), file=sys.stderr,
          flush=True)
    sub = qsd.Subspace(w.keys, w.ops.n_qubits, max_load=max_load)
    kw = {} if group_order == "default" else {"order_by_mask": group_order == "mask",
                                                "order_by_parts": group_order == "parts"}
    op = qsd.operator_from_termlist(w.ops, **kw)
    if group_order == "default":
        group_order = "parts" if w.ops.fermionic else "weight"

    H = qsd.SubspaceHamiltonian(sub, op)
    N, W = sub.N, sub.W
    # structural nonzeros (CSR count pass) and work counters, outside the timed region
    indptr = torch.empty(N + 1, dtype=torch.int64, device="cuda")
    nnz_c = ctypes.c_int64()
    qsd._check(qsd.lib().qsd_csr_build(H.handle, qsd._ptr(indptr), None, None, qsd.INDEX_I64,
                                       qsd.C128 if H.is_complex else qsd.F64, ctypes.byref(nnz_c), qsd._stream()))
    nnz = nnz_c.value
    probes, hits = H.work_counts()
    del indptr
    dt = torch.float64 if dtype_name == "f64" else torch.float32
    tune = None
    if schedule == "auto":
        if split > 0:
            sub.rehash(max_load, split)
        tune = H.autotune(nvec=nvec, dtype=dt, reps=3, load=max_load == 0.0, split=split < 0)
        print("# autotuner: %s" % json.dumps(tune), file=sys.stderr, flush=True)
    else:
        if split > 0 or max_load:
            sub.rehash(max_load, max(split, 0))
        H.schedule = int(schedule)
    sched = H.schedule
    hsplit, exact, product = sub.hash_info()
    setup_s = time.perf_counter() - t_setup
    print("# setup %.1f s: N=%d nnz=%d probes=%d hits=%d groups=%d" % (setup_s, N, nnz, probes, hits, op.n_groups),
          file=sys.stderr, flush=True)

    esz = 8 if dtype_name == "f64" else 4
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    x = torch.rand((N, nvec), dtype=dt, device="cuda", generator=g).squeeze(1)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        H.matvec(x, out=y)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        H.matvec(x, out=y)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [e0.elapsed_time(e1) for e0, e1 in evs]
    k_avg = float(np.mean(kms))
    ms_per_step = wall * 1e3 / steps
    balg = algorithmic_bytes(N, W, probes, hits, nvec, esz)
    achieved = balg / (k_avg / 1e3) / 1e9
    print("# SpMV: %.4f ms/step wall, kernel avg %.4f ms (min %.4f), %.1f GB/s algorithmic" %
          (ms_per_step, k_avg, min(kms), achieved), file=sys.stderr, flush=True)
    res = {
        "value": nnz * nvec / (ms_per_step / 1e3),
        "ms_per_step": ms_per_step,
        "config": {"workload": w.name, "n_qubits": w.ops.n_qubits, "subspace_dim": N, "nnz": nnz,
                   "groups": op.n_groups, "terms": op.n_terms, "nvec": nvec, "kernel": "k_matvec",
                   "schedule": sched, "hash_capacity": sub.capacity, "part_filter_split": hsplit,
                   "exact_slots": exact, "product_map": product, "group_order": group_order,
                   "autotune": tune},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic(w.name, dtype_name, nvec, sub.capacity),
                     "bytes_per_launch": balg, "kernel_ms": k_avg, "kernel_ms_min": min(kms),
                     "kernel_source_digest": kernel_digest()},
        "roofline_issue": None,
        "work": {"probes": probes, "hits": hits, "evaluations": N * op.n_groups,
                 "probes_per_s": probes / (k_avg / 1e3), "evaluations_per_s": N * op.n_groups / (k_avg / 1e3)},
    }
    # the instruction-issue roofline, from the profiled VALU instruction count of this kernel
    valu = stored_traffic(w.name, dtype_name, nvec, sub.capacity, key="valu_insts_per_launch")
    if valu is not None:
        res["roofline_issue"] = {"bound": "valu_issue", "achieved": valu / (k_avg / 1e3), "peak": VALU_ISSUE_PEAK,
                                 "unit": "wave instructions/s", "frac": valu / (k_avg / 1e3) / VALU_ISSUE_PEAK,
                                 "insts_per_launch": valu}
    if solve:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, _, info = H.lanczos(tol=1e-10, max_iter=300, v0="uniform", raise_on_nonconv=False)
        solve_s = time.perf_counter() - t0
        res["ground_state"] = {"energy": e, "solve_s": solve_s, "iterations": info["iterations"],
                               "converged": bool(info["converged"]), "ritz_residual": info["ritz_residual"]}
        print("# ground state %.12f in %.3f s (%d iterations)" % (e, solve_s, info["iterations"]), file=sys.stderr,
              flush=True)
    del H, op, sub, x, y
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
