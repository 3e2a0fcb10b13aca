#!/usr/bin/env python3
"""Benchmark: matrix-free subspace-Hamiltonian SpMV on one MI355X.

A step is one matrix-free SpMV ``y = H_S x`` over the whole subspace (diagonal, group scan,
ladder-integer ranges, hash probes, projector refinement, accumulation), with the subspace,
hash table, operator tables and vectors resident in HBM.  The default workload is the 2D XXZ
model on the open 6x6 grid (Jxy = 1, Jz = 0.8, ladder form) over 2^20 distinct weight-18
bit-strings, in FP64.

Output: one JSON line.  ``value`` = stored matrix elements (structural nonzeros of H_S)
processed per second of SpMV.  ``roofline`` prices the SpMV kernel's algorithmic bytes
against the 8 TB/s HBM peak.  ``cpu_baseline`` times the CPU oracle (term-by-term, binary
search) on the host cores on the same input.  Extra keys report the ground-state solve time
(GPU Lanczos, FP64) and the work counters.
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
KERNEL_SOURCES = ["paper_2603_18731_amd/csrc/engine.h", "paper_2603_18731_amd/csrc/matvec.h",
                  "paper_2603_18731_amd/csrc/device.h"]
# the SpMV kernels and their launch in ham.hip (the rest of that file is host code)
KERNEL_FUNCTIONS = ("paper_2603_18731_amd/csrc/ham.hip", ("void k_matvec(", "void launch_mv("))


def kernel_digest():
    """Digest of the SpMV kernel's sources (ties a stored counter profile to the code)."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    path, names = KERNEL_FUNCTIONS
    with open(os.path.join(ROOT, path)) as fh:
        text = fh.read()
    for name in names:
        i = text.index(name)
        j = text.index("\n}\n", i)  # end of the function body
        h.update(text[i:j].encode())
    return h.hexdigest()[:16]


def stored_traffic(workload, dtype, nvec, capacity):
    """HBM bytes per SpMV launch from the committed counter profile of this workload, or None
    when there is none, it was taken on other kernel sources or with another hash-table size.
    The profile records FETCH_SIZE and WRITE_SIZE per dispatch (KiB) and the factors that scale
    them to the bytes a plain copy of known size moves."""
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
    return float(vals["hbm_bytes_per_launch"])


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
    """Bytes the method must move per SpMV: per row the key (8W), its hash (8), the diagonal
    (8), x_i and y_i (2 * esz * nvec); per probe one 8-byte slot; per hit the key compare (8W)
    and the gathered x_j (esz * nvec)."""
    return N * (8 * W + 16 + 2 * esz * nvec) + probes * 8 + hits * (8 * W + esz * nvec)


def make_workload(name):
    import workloads as wl

    if name == "xxz6x6":
        w = wl.c2_xxz6x6()
    elif name == "tfim12":
        w = wl.c1_tfim12()
    elif name == "fermi16":
        w = wl.c3_molecular()
    elif name == "heavyhex200":
        w = wl.c4_heavy_hex()
    else:
        raise SystemExit("unknown workload %s" % name)
    return w


def cpu_baseline(w, nnz_total, budget_s=12.0):
    """Time the CPU oracle's SpMV over all rows (repeated until ~budget_s) or, for large
    workloads, over a row sample scaled to the full matrix."""
    import numpy as np

    from oracle import rowwise as orw
    from oracle import subspace as osub

    ck = osub.canonical_keys(w.keys)
    N = ck.shape[0]
    rng = np.random.default_rng(0)
    x = rng.normal(size=N)
    threads = orw.max_threads()
    # probe the cost on a small sample first
    rows = np.sort(rng.choice(N, size=min(N, 2000), replace=False))
    t0 = time.perf_counter()
    orw.matvec_c(ck, w.ops, x, rows)
    per_row = (time.perf_counter() - t0) / len(rows)
    if per_row * N <= budget_s / 2:
        reps, t_total = 0, 0.0
        while t_total < budget_s and reps < 50:
            t0 = time.perf_counter()
            orw.matvec_c(ck, w.ops, x)
            t_total += time.perf_counter() - t0
            reps += 1
        t_mv = t_total / reps
        sample = "all %d rows, %d repetitions" % (N, reps)
    else:
        nrow = max(1000, min(N, int(budget_s / per_row)))
        rows = np.sort(rng.choice(N, size=nrow, replace=False))
        t0 = time.perf_counter()
        orw.matvec_c(ck, w.ops, x, rows)
        t_mv = (time.perf_counter() - t0) * N / nrow
        sample = "%d of %d rows, time scaled to all rows" % (nrow, N)
    return {"value": nnz_total / t_mv, "unit": "matrix elements/s", "cores": threads, "kind": "oracle",
            "sample": sample, "matvec_s": t_mv}


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

    # FIFO baseline: plain FP64 single-vector Lanczos, one request at a time
    service = np.zeros(n)
    e_fifo = np.zeros(n)
    iters_fifo = np.zeros(n, dtype=np.int64)
    for i, H in enumerate(hams):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, _, info = H.lanczos(tol=1e-10, max_iter=max_iter, v0="uniform", raise_on_nonconv=False)
        service[i] = time.perf_counter() - t0
        e_fifo[i], iters_fifo[i] = e, info["iterations"]
        if (i + 1) % 32 == 0:
            print("# fifo %d/%d solved (%.1f s of service so far)" % (i + 1, n, service.sum()), file=sys.stderr,
                  flush=True)
    mu_fifo = n / service.sum()

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
    for f in (0.7, 0.9):
        arr = serve.poisson_arrivals(n, f * mu, seed=5 + int(f * 10))
        out_open["lambda_%.1f_mu" % f] = dict(run(arr, "open loop %.1f mu" % f), rate_per_s=f * mu)
        fifo_open["lambda_%.1f_mu" % f] = serve.percentiles(serve.fifo_latencies(arr, service))
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
    }
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
    for block in (1, 8):
        e64 = out["energy_f64_b%d" % block]
        out["energy_rel_err_f32_b%d" % block] = abs(out["energy_f32_b%d" % block] - e64) / abs(e64)
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
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="xxz6x6")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--nvec", type=int, default=1)
    ap.add_argument("--max-load", type=float, default=0.0, help="hash load factor (0 = library default)")
    ap.add_argument("--schedule", default="auto", help="SpMV schedule bits, or 'auto' for the autotuner")
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
        import paper_2603_18731_amd as qsd

        for kib in (256, 1024, 2048, 4096, 8192, 32768, 131072, 524288, 1048576):
            for ilp in (1, 2, 4, 8):
                r = qsd.device_gather_rate(kib << 10, ilp)
                print(json.dumps({"buffer_kib": kib, "ilp": ilp, "loads_per_s": r}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library does not shard the subspace SpMV across "
              "GPUs (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2603_18731_amd as qsd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    w = make_workload(args.workload)
    print("# workload %s: %d strings, %d qubits" % (w.name, w.keys.shape[0], w.ops.n_qubits), file=sys.stderr,
          flush=True)
    sub = qsd.Subspace(w.keys, w.ops.n_qubits, max_load=args.max_load)
    op = qsd.operator_from_termlist(w.ops)
    H = qsd.SubspaceHamiltonian(sub, op)
    N, W = sub.N, sub.W
    # structural nonzeros (CSR count pass) and work counters, outside the timed region
    indptr = torch.empty(N + 1, dtype=torch.int64, device="cuda")
    import ctypes

    nnz_c = ctypes.c_int64()
    qsd._check(qsd.lib().qsd_csr_build(H.handle, qsd._ptr(indptr), None, None, qsd.INDEX_I64,
                                       qsd.C128 if H.is_complex else qsd.F64, ctypes.byref(nnz_c), qsd._stream()))
    nnz = nnz_c.value
    probes, hits = H.work_counts()
    del indptr
    dt = torch.float64 if args.dtype == "f64" else torch.float32
    tune = None
    if args.schedule == "auto":
        tune = H.autotune(nvec=args.nvec, dtype=dt, reps=3, load=args.max_load == 0.0)
        print("# autotuner: %s" % json.dumps(tune), file=sys.stderr, flush=True)
    else:
        H.schedule = int(args.schedule)
    sched = H.schedule
    setup_s = time.perf_counter() - t_setup
    print("# setup %.1f s: N=%d nnz=%d probes=%d hits=%d groups=%d" % (setup_s, N, nnz, probes, hits, op.n_groups),
          file=sys.stderr, flush=True)

    esz = 8 if args.dtype == "f64" else 4
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    x = torch.rand((N, args.nvec), dtype=dt, device="cuda", generator=g).squeeze(1)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        H.matvec(x, out=y)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        H.matvec(x, out=y)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [e0.elapsed_time(e1) for e0, e1 in evs]
    k_avg = float(np.mean(kms))
    ms_per_step = wall * 1e3 / args.steps
    value = nnz * args.nvec / (ms_per_step / 1e3)
    balg = algorithmic_bytes(N, W, probes, hits, args.nvec, esz)
    achieved = balg / (k_avg / 1e3) / 1e9
    print("# SpMV: %.4f ms/step wall, kernel avg %.4f ms (min %.4f), %.1f GB/s algorithmic" %
          (ms_per_step, k_avg, min(kms), achieved), file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "matrix elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "n_qubits": w.ops.n_qubits, "subspace_dim": N, "nnz": nnz,
                   "groups": op.n_groups, "terms": op.n_terms, "nvec": args.nvec,
                   "kernel": "k_matvec",
                   "schedule": sched, "hash_capacity": sub.capacity, "autotune": tune},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic(w.name, args.dtype, args.nvec, sub.capacity), "bytes_per_launch": balg,
                     "kernel_ms": k_avg, "kernel_source_digest": kernel_digest()},
        "work": {"probes": probes, "hits": hits, "evaluations": N * op.n_groups,
                 "probes_per_s": probes / (k_avg / 1e3), "evaluations_per_s": N * op.n_groups / (k_avg / 1e3)},
    }
    if not args.no_solve:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, _, info = H.lanczos(tol=1e-10, max_iter=300, v0="uniform", raise_on_nonconv=False)
        solve_s = time.perf_counter() - t0
        out["ground_state"] = {"energy": e, "solve_s": solve_s, "iterations": info["iterations"],
                               "converged": bool(info["converged"]), "ritz_residual": info["ritz_residual"]}
        print("# ground state %.12f in %.3f s (%d iterations)" % (e, solve_s, info["iterations"]), file=sys.stderr,
              flush=True)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, nnz * args.nvec)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        print("# cpu oracle %.3f s per SpMV on %d threads" % (cb["matvec_s"], cb["cores"]), file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
