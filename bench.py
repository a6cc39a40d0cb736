"""Benchmark of the Block Krylov hot path on one MI355X.

A step is one whole solve (sketch, Krylov products, projection,
CholeskyQR, M = W^T W -- or the block-tridiagonal T of block Lanczos with
--method lanczos --, the eigen-solve, Z = Q U_k) on one synthetic input
already resident in HBM.  Default workload: the term-document CSR matrix
(11000 x 130000, ~1.47M nonzeros, log-normal row lengths, Zipf(1.1) terms,
log(1+tf)*idf values), k = 20, q = 10, implicit row centring, FP32.

Metric: GB/s of the Krylov block products A.X / A^T.Y, i.e. the algorithmic
bytes those products must move in one solve divided by the time of the whole
solve.  The roofline object reports the dominant product kernel alone:
algorithmic bytes per launch / its average launch time (HIP events recorded
on the solve's stream inside the timed steps) against the 8 TB/s HBM peak.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       [--workload csr2|dense1|dense3|dense4|dense5] [--precision plain|bf16|fp8]
       [--method bki|lanczos] [--time-to-eps] [--metrics-q Q]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = ("Krylov A·X/Aᵀ·Y GB/s or TFLOP/s & time-to-ε "
          "(BF16/FP8 vs FP32), 1 GPU")
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFS = 157.3
DESCR = {
    "csr2": "term-document CSR 11000x130000 (~1.47M nnz, log-normal rows, Zipf(1.1) "
            "terms, log(1+tf)*idf), k=20, q=10, implicit row centring",
    "dense1": "dense planted sigma_i=i^-1/2 2000x1000, k=10, q=8, FP64",
    "dense3": "dense planted sigma_i=exp(-i/200)+1e-3 (+1e-4 noise) 65536x16384, k=100, q=12",
    "dense4": "dense planted sigma_i=1/i 8192x4096, k=32, q=10",
    "dense5": "dense planted sigma_i=i^-0.8 131072x32768, k=256, q=8",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------- inputs --
def make_csr(w):
    rp, ci, va = workloads.term_document_csr(w.n, w.d, w.seed_matrix)
    return rp, ci, va


def csr_product_bytes(n, d, nnz, k):
    """Algorithmic bytes of one A.X and one A^T.Y (CSR of A^T): values and
    column ids once, row pointers once, the dense input block once, the
    output block once."""
    ax = nnz * 8 + (n + 1) * 4 + d * k * 4 + n * k * 4
    aty = nnz * 8 + (d + 1) * 4 + n * k * 4 + d * k * 4
    return ax, aty


def dense_product_bytes(n, d, k, a_bytes, x_bytes):
    ax = n * d * a_bytes + d * k * x_bytes + n * k * x_bytes
    aty = n * d * a_bytes + n * k * x_bytes + d * k * x_bytes
    return ax, aty


def source_sha(names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_1504_05477_amd", "csrc", nm), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_key, sha):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel, if it was taken on the current source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_key}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                key, v = line.split(":", 1)
                vals[key.strip()] = v.strip()
    if vals.get("source_sha") != sha:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---------------------------------------------------------------- main --
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="csr2", choices=sorted(workloads.WORKLOADS))
    ap.add_argument("--precision", default="plain", choices=["plain", "bf16", "fp8"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--breakdown", action="store_true", help="phase times to stderr")
    ap.add_argument("--method", default="bki", choices=["bki", "lanczos", "si"],
                    help="Rayleigh-Ritz matrix: W^T W (Algorithm 2) or the block-tridiagonal "
                         "T of the block Lanczos recurrence (Section 4.2); or simultaneous "
                         "iteration (Algorithm 1)")
    ap.add_argument("--block-size", type=int, default=0, metavar="P",
                    help="block width p >= k (oversampling, Section 6); 0: p = k")
    ap.add_argument("--time-to-eps", action="store_true",
                    help="dense workloads: for each eps in 1e-1, 1e-2, 1e-3 the smallest q whose "
                         "per-vector error (eq. 3, planted spectrum, measured on the GPU) is at "
                         "most eps, and the time of one solve at that q")
    ap.add_argument("--metrics-q", type=int, default=4, metavar="Q",
                    help="depth of the GPU spectral-residual estimate of the error measures "
                         "taken after the timed steps (-1: skip them)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (the reference "
                         "kernel that scales the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1504_05477_amd as bk

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    bk.load()
    dev = torch.device("cuda:0")
    w = workloads.WORKLOADS[args.workload]
    k, q = w.k, w.q
    t_gen = time.perf_counter()
    host_inputs = {}
    prep_ms = {}
    if w.kind == "csr":
        rp, ci, va = make_csr(w)
        host_inputs = {"rp": rp, "ci": ci, "va": va}
        g_rp = torch.from_numpy(rp).to(dev)
        g_ci = torch.from_numpy(ci).to(dev)
        g_va = torch.from_numpy(va).to(dev)
        nnz = int(ci.size)
        bx, by = csr_product_bytes(w.n, w.d, nnz, args.block_size or k)
        dtype = "f32"
        # CSR of A^T: an input layout built once on the GPU (as a caller
        # solving repeatedly would), timed on its own, outside the steps
        tr = bk.csr_transpose(g_rp, g_ci, g_va, w.d)
        torch.cuda.synchronize()
        t0p = time.perf_counter()
        for _ in range(3):
            tr = bk.csr_transpose(g_rp, g_ci, g_va, w.d)
        torch.cuda.synchronize()
        prep_ms["csr_transpose"] = round((time.perf_counter() - t0p) * 1e3 / 3, 4)

        def step(timing):
            return bk.svd_csr(g_rp, g_ci, g_va, w.n, w.d, k, q, seed=w.seed_sketch,
                              center=w.center, transpose=tr, timing=timing,
                              method=args.method, block_size=args.block_size)

        def error_measures(Z, qs):
            return bk.error_metrics_csr(g_rp, g_ci, g_va, w.n, w.d, Z, q_spec=qs,
                                        seed=w.seed_sketch + 1, center=w.center, transpose=tr)
        kern_src = ["csr.hip"]
        kern_names = {"ax": "csr_product_kernel (A.X, CSR of A)",
                      "aty": "csr_product_kernel (A^T.Y, CSR of A^T)"}
    else:
        sv = workloads.spectrum(w.spectrum, min(w.n, w.d))
        if w.n * w.d <= 4_000_000:
            A64 = workloads.planted_dense(w.n, w.d, sv, w.seed_matrix)
            host_inputs = {"A": A64}
            A = torch.from_numpy(A64).to(dev)
            if w.dtype != "f64":
                A = A.float()
        else:
            A = workloads.planted_dense_torch(w.n, w.d, sv, w.seed_matrix, device=dev,
                                              noise=w.noise, noise_seed=w.seed_noise)
        if w.dtype == "f64":
            A = A.double()
        kw = {}
        a_bytes = A.element_size()
        dtype = "f64" if A.dtype == torch.float64 else "f32"
        if args.precision in ("bf16", "fp8"):
            # the low-precision copy is made once, outside the timed steps
            torch.cuda.synchronize()
            t0p = time.perf_counter()
            if args.precision == "bf16":
                A_in = bk.quantize(A, "bf16")
                kw = {"A_master": A}
                a_bytes, dtype = 2, "bf16"
            else:
                A_in, sc = bk.quantize(A, "fp8")
                kw = {"A_master": A, "a_scales": sc}
                a_bytes, dtype = 1, "fp8"
            torch.cuda.synchronize()
            prep_ms["quantize"] = round((time.perf_counter() - t0p) * 1e3, 4)
        else:
            A_in = A
        x_bytes = 8 if A.dtype == torch.float64 else 4
        bx, by = dense_product_bytes(w.n, w.d, args.block_size or k, a_bytes, x_bytes)

        def step(timing):
            return bk.svd_dense(A_in, k, q, seed=w.seed_sketch, timing=timing,
                                method=args.method, block_size=args.block_size, **kw)

        def error_measures(Z, qs):
            return bk.error_metrics_dense(A, Z.to(A.dtype).contiguous(), q_spec=qs,
                                          seed=w.seed_sketch + 1)

        def solve_q(qq):
            return bk.svd_dense(A_in, k, qq, seed=w.seed_sketch, **kw)

        def per_vector(Z):
            m = bk.error_metrics_dense(A, Z.to(A.dtype).contiguous(),
                                       sigma_true=sv[:k + 1], q_spec=0, seed=w.seed_sketch + 1)
            return m.values["per_vector"]
        kern_src = ["gemm.hip", "gemm_mfma.hip"]
        kern_names = {"ax": "A.X product (operand pack + product kernel)",
                      "aty": "A^T.Y product (operand pack + product kernel + split reduction)"}
    torch.cuda.synchronize()
    log(f"inputs ready in {time.perf_counter() - t_gen:.1f}s ({args.workload})")

    # The last n_ev timed steps record events around the product phases (the
    # roofline kernel's launch durations); an event between two kernels
    # stalls the queue (~4 us), so the other timed steps run without them.
    # The per-phase breakdown comes from extra steps after the timed region.
    timed_phases = ("ax", "aty")
    n_ev = min(2, args.steps)
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step(timed_phases if i >= args.steps - n_ev else False)
        infos.append(r.info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    bytes_per_solve = (q + 1) * (bx + by)
    value = bytes_per_solve / (ms_step * 1e-3) / 1e9
    nbd = 2
    full = [step(True).info for _ in range(nbd)]
    torch.cuda.synchronize()

    def tot(key, what="ms"):
        return sum(float(i[what][key]) for i in infos[-n_ev:])
    ph = {p: sum(float(i["ms"][p]) for i in full) / nbd for p in full[0]["ms"]}
    if args.breakdown:
        log("phase ms/step: " + ", ".join(f"{p}={v:.3f}" for p, v in ph.items()))
        log(f"launches/step: {full[0]['launches']}")
    dom = "ax" if tot("ax") >= tot("aty") else "aty"
    if w.kind == "csr":
        # one product kernel per launch in these phases (the combine and
        # centring kernels are timed in phases of their own)
        nl = tot(dom, "launches")
    else:
        # a dense product is a short sequence of kernels (operand packing,
        # the MFMA or vector product, the split reduction): rate per product
        nl = n_ev * (infos[-1]["q_eff"] + 1)
    avg_ms = tot(dom) / max(nl, 1)
    per_launch = bx if dom == "ax" else by
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    sha = source_sha(kern_src)
    kernel_key = f"{'csr_product' if w.kind == 'csr' else 'dense_product'}_{dom}_{args.workload}"
    traffic = read_traffic(kernel_key, sha)
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": kern_names[dom],
            "avg_launch_ms": round(avg_ms, 5), "event_steps": n_ev,
            "algorithmic_bytes_per_launch": int(per_launch), "source_sha": sha}
    if w.kind == "dense" and args.precision == "plain":
        flops = 2.0 * w.n * w.d * (args.block_size or k)
        tf = flops / (avg_ms * 1e-3) / 1e12
        if flops / per_launch > FP32_PEAK_TFS * 1e12 / (HBM_PEAK_GBS * 1e9):
            roof.update({"bound": "mfma", "achieved": round(tf, 3),
                         "peak": FP32_PEAK_TFS if dtype == "f32" else 78.6,
                         "unit": "TFLOP/s", "frac": round(tf / (FP32_PEAK_TFS if dtype == "f32" else 78.6), 4)})
        roof["avg_ms_is"] = "per product"

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {DESCR[args.workload]}",
                   "n": w.n, "d": w.d, "k": k, "q": q,
                   "precision": args.precision, "method": args.method,
                   "block_size": args.block_size or k,
                   "product_bytes_per_solve": int(bytes_per_solve)},
        "roofline": roof,
        "phases_ms_per_step": {p: round(v, 4) for p, v in ph.items()},
        "products_all_kernels": products_all_kernels(ph, infos[-1]["q_eff"], bx, by),
        "input_prep_ms_untimed": prep_ms,
        "q_eff": infos[-1]["q_eff"],
        "jacobi_sweeps": infos[-1]["jacobi_sweeps"],
    }

    if args.metrics_q >= 0:
        out["error_measures"] = gpu_error_measures(error_measures, r.Z, args.metrics_q)
    if args.time_to_eps:
        if w.kind == "dense":
            out["time_to_eps"] = time_to_eps(solve_q, per_vector, q)
        else:
            out["time_to_eps"] = {"skipped": "needs the true spectrum (planted dense inputs)"}

    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity"] = cpu_baseline(args, w, host_inputs, r,
                                                          bytes_per_solve)
    print(json.dumps(out), flush=True)


def gpu_error_measures(fn, Z, qs):
    """eqs. (1)-(3) quantities of the last solve's Z on the GPU (Section 3):
    ||Abar||_F^2, the Frobenius residual (Pythagoras), the spectral residual
    (block Krylov on (I - Z Z^T) Abar, depth qs); no true spectrum at this
    size, so the ratios are not formed.  Wall time of one call (it
    synchronizes), after a warm-up call."""
    import torch
    fn(Z, qs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = fn(Z, qs)
    ms = (time.perf_counter() - t0) * 1e3
    v = m.values
    return {"fro2": v["fro2"], "resid_fro": v["resid_fro"], "resid_spec": v["resid_spec"],
            "captured_fro2": v["captured_fro2"], "q_spec": qs, "ms": round(ms, 3),
            "status": m.status}


def time_to_eps(solve_q, per_vector, q_max, eps_list=(1e-1, 1e-2, 1e-3), reps=3):
    """Time-to-eps (the paper's per-vector error, eq. 3, against the planted
    spectrum, Section 7): for q = 0 .. q_max the per-vector error of one
    solve's Z (error measures on the GPU) and the median wall time of `reps`
    solves after one warm-up; for each eps the smallest q reaching it."""
    import torch
    rows = []
    for qq in range(0, q_max + 1):
        solve_q(qq)
        torch.cuda.synchronize()
        ts = []
        res = None
        for _ in range(reps):
            t0 = time.perf_counter()
            res = solve_q(qq)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        rows.append({"q": qq, "per_vector": per_vector(res.Z), "ms": round(sorted(ts)[reps // 2], 4)})
    out = {"sweep": rows}
    for eps in eps_list:
        hit = next((r for r in rows if r["per_vector"] <= eps), None)
        out[f"{eps:g}"] = ({"q": hit["q"], "ms": hit["ms"]} if hit else "not reached")
    return out


def products_all_kernels(ph, q_eff, bx, by):
    """Rate of the block products counting every kernel they launch (CSR:
    product, combine of rows cut into pieces, centring sums)."""
    nprod = q_eff + 1
    ms = ph["ax"] + ph["aty"] + ph.get("long", 0.0) + ph.get("center", 0.0)
    per = ms / (2 * nprod)
    return {"ms_per_product": round(per, 5),
            "GBps": round((bx + by) / 2 / (per * 1e-3) / 1e9, 2),
            "products_per_step": 2 * nprod}


def copy_calibration(mib):
    """Plain device-to-device copies of a known size: under rocprofv3 --pmc
    the FETCH_SIZE / WRITE_SIZE they read give the factor from counter KiB
    to bytes moved (each copy reads and writes mib MiB)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": n * 4,
                      "copy_bytes_written_per_launch": n * 4, "launches": 5}), flush=True)


def cpu_baseline(args, w, host, res, bytes_per_solve):
    """The oracle, as it stands, on the host cores: whole solves of the same
    input repeated for about --cpu-seconds (the sample), in the same unit."""
    import scipy.sparse as sp
    from threadpoolctl import threadpool_info

    from oracle import bki, metrics, philox

    k, q = w.k, w.q
    pw = args.block_size or k
    Pi = philox.gaussian(w.seed_sketch, w.d, pw)
    if w.kind == "csr":
        A = sp.csr_matrix((host["va"].astype(np.float64), host["ci"], host["rp"]),
                          shape=(w.n, w.d))
        Pi = Pi.astype(np.float32).astype(np.float64)
        tau = 1e-5
    elif "A" in host:
        A = host["A"] if w.dtype == "f64" else host["A"].astype(np.float32).astype(np.float64)
        if w.dtype != "f64":
            Pi = Pi.astype(np.float32).astype(np.float64)
        tau = 1e-11 if w.dtype == "f64" else 1e-5
    else:
        return ({"value": None, "unit": "GB/s", "cores": 0, "kind": "oracle",
                 "sample": "skipped: matrix generated on the GPU only"}, None)
    times = []
    ref = None
    t_end = time.perf_counter() + args.cpu_seconds
    while time.perf_counter() < t_end or not times:
        t0 = time.perf_counter()
        # the oracle route of the method timed on the GPU
        if args.method == "si":
            ref = bki.simultaneous_iteration(A, Pi, k, q, center=w.center)
        elif args.method == "lanczos":
            ref = bki.block_lanczos(A, Pi, k, q, center=w.center, tau=tau)[0]
        else:
            ref = bki.block_krylov(A, Pi, k, q, center=w.center, tau=tau)
        times.append(time.perf_counter() - t0)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    per = float(np.median(times))
    base = {"value": round(bytes_per_solve / per / 1e9, 4), "unit": "GB/s",
            "cores": int(threads), "kind": "oracle",
            "sample": f"{len(times)} whole solves of the same input "
                      f"(median {per * 1e3:.1f} ms/solve, NumPy/SciPy float64; sparse "
                      f"products single-threaded, dense BLAS on {threads} threads)",
            "ms_per_solve": round(per * 1e3, 2)}
    Zg = res.Z.double().cpu().numpy()
    sg = res.sigma.cpu().numpy()
    rel = float(np.max(np.abs(sg - ref.sigma) / ref.sigma))
    j = 0   # widest leading subspace with relative Ritz gap >= 1e-2
    for jj in range(1, min(k, len(ref.theta) - 1) + 1):
        if (ref.theta[jj - 1] - ref.theta[jj]) / ref.theta[0] >= 1e-2:
            j = jj
    ang = metrics.principal_angle(ref.Z[:, :j], Zg[:, :j]) if j else None
    parity = {"ritz_rel_max": rel, "principal_angle_rad": ang, "gap_separated_j": j,
              "angle_at_k_rad": metrics.principal_angle(ref.Z, Zg)}
    return base, parity


if __name__ == "__main__":
    main()
