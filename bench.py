"""Benchmark of the Block Krylov hot path on one MI355X.

A step is one whole solve (sketch, Krylov products, projection,
CholeskyQR, M = W^T W -- or the block-tridiagonal T of block Lanczos with
--method lanczos --, the eigen-solve, Z = Q U_k) on one synthetic input
already resident in HBM.

Default workload: the large dense matrix, 131072 x 32768 with planted
singular values sigma_i = i^-0.8, k = 256, q = 8.  The plain FP32 path is
the timed line; the FP8 e4m3 copy (128 x 128 tile scales, one FP32
correction pass on the FP32 master) is timed in the same run on the same
matrix and reported beside it with its speedup.  Both results are compared
with the float64 oracle (Algorithm 2 run in the coordinates of the planted
factors) and the oracle's block products are timed on the host cores.

Metric: throughput of the Krylov block products A.X / A^T.Y over whole
solves -- TFLOP/s when the product is bound by the matrix cores (FP32 with
arithmetic intensity above the FP32 ridge), GB/s of algorithmic bytes
otherwise.  The roofline object reports the dominant product alone (HIP
events recorded on the solve's stream inside the timed steps).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       [--workload dense5|dense3|dense4|dense1|csr2] [--precision plain|bf16|fp8]
       [--compare auto|none|bf16|fp8] [--method bki|lanczos|si] [--time-to-eps]
       [--metrics-q Q] [--no-parity] [--no-cpu-baseline]
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
PEAK_TFS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "fp8": 5000.0}
# FP32 products as three BF16 limbs: six BF16 matrix-core products per FP32
# product, so the FP32-equivalent peak is the dense BF16 peak over six
LIMB_PEAK_TFS = PEAK_TFS["bf16"] / 6.0


def f32_peak(args):
    """(peak TFLOP/s, basis) of the FP32 products in this run."""
    if getattr(args, "fp32_products", "limbs") == "limbs":
        return LIMB_PEAK_TFS, "dense BF16 2.5 PFLOP/s / 6 limb products"
    return PEAK_TFS["f32"], "FP32 matrix cores 157.3 TFLOP/s"
DESCR = {
    "csr2": "term-document CSR 11000x130000 (~1.47M nnz, log-normal rows, Zipf(1.1) "
            "terms, log(1+tf)*idf), k=20, q=10, implicit row centring",
    "dense1": "dense planted sigma_i=i^-1/2 2000x1000, k=10, q=8, FP64",
    "dense3": "dense planted sigma_i=exp(-i/200)+1e-3 (+1e-4 noise) 65536x16384, k=100, q=12",
    "dense4": "dense planted sigma_i=1/i 8192x4096, k=32, q=10",
    "dense5": "dense planted sigma_i=i^-0.8 131072x32768, k=256, q=8",
}
# low-precision form timed beside the plain FP32 path (--compare auto)
AUTO_COMPARE = {"dense5": "fp8", "dense3": "bf16"}


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


def value_unit(kind, dtype, n, d, pw, a_bytes, peak=None):
    """TFLOP/s for FP32 / FP64 dense products above the ridge of their
    matrix-core peak (flops per byte), GB/s otherwise."""
    if kind != "dense" or dtype not in ("f32", "f64"):
        return "GB/s"
    ai = 2.0 * n * d * pw / (n * d * a_bytes)
    ridge = (peak or PEAK_TFS[dtype]) * 1e12 / (HBM_PEAK_GBS * 1e9)
    return "TFLOP/s" if ai > ridge else "GB/s"


def rate(unit, bytes_, flops, ms):
    if unit == "TFLOP/s":
        return flops / (ms * 1e-3) / 1e12
    return bytes_ / (ms * 1e-3) / 1e9


# --------------------------------------------------------------- legs --
def timed_leg(step, steps, warmup):
    """`warmup` untimed solves, `steps` timed ones (the last two record HIP
    events around the product phases only: an event between two kernels
    stalls the queue for ~4 us), then two solves with events on every phase
    for the breakdown."""
    import torch
    timed_phases = ("ax", "aty")
    n_ev = min(2, steps)
    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    r = None
    for i in range(steps):
        r = step(timed_phases if i >= steps - n_ev else False)
        infos.append(r.info)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    full = [step(True).info for _ in range(2)]
    torch.cuda.synchronize()
    ph = {p: sum(float(i["ms"][p]) for i in full) / len(full) for p in full[0]["ms"]}
    return {"ms": ms, "infos": infos, "n_ev": n_ev, "phases": ph, "launches": full[0]["launches"],
            "last": r}


def dominant_product(leg, kind):
    """(phase, average ms per launch) of the larger product phase over the
    event-timed steps."""
    infos, n_ev = leg["infos"], leg["n_ev"]

    def tot(key, what="ms"):
        return sum(float(i[what][key]) for i in infos[-n_ev:])
    dom = "ax" if tot("ax") >= tot("aty") else "aty"
    if kind == "csr":
        # one product kernel per launch in these phases (the combine and
        # centring kernels are timed in phases of their own)
        nl = tot(dom, "launches")
    else:
        # a dense product is a short sequence of kernels (operand packing,
        # the MFMA or vector product, the split reduction): rate per product
        nl = n_ev * (infos[-1]["q_eff"] + 1)
    return dom, tot(dom) / max(nl, 1)


# ---------------------------------------------------------------- main --
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dense5", choices=sorted(workloads.WORKLOADS))
    ap.add_argument("--precision", default="plain", choices=["plain", "bf16", "fp8"])
    ap.add_argument("--compare", default="auto", choices=["auto", "none", "bf16", "fp8"],
                    help="low-precision copy timed beside the plain path on the same matrix "
                         "(auto: FP8 for dense5, BF16 for dense3, none otherwise)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the comparison with the float64 oracle")
    ap.add_argument("--breakdown", action="store_true", help="phase times to stderr")
    ap.add_argument("--fp32-products", default="limbs", choices=["limbs", "cores"],
                    help="FP32 block products as three BF16 limbs on the BF16 matrix cores "
                         "(limbs) or on the FP32 matrix cores (cores)")
    ap.add_argument("--csr-gather", default="default", choices=["default", "inplace", "staged"],
                    help="CSR workloads: gather the right-hand block's rows from the Krylov "
                         "block (inplace) or from a copy with 128-byte-aligned rows (staged)")
    ap.add_argument("--lowp-layout", default="both", choices=["both", "rows"],
                    help="low-precision leg: also hold the copy transposed, so that the "
                         "A^T Y products read it row by row (both), or A only (rows)")
    ap.add_argument("--input", default="planted", choices=["planted", "gaussian"],
                    help="dense workloads: the planted matrix of the workload, or a seeded "
                         "N(0, 1/d) matrix of the same shape built without factorizations "
                         "(for profiler counter runs; no parity or CPU baseline)")
    ap.add_argument("--method", default="bki", choices=["bki", "lanczos", "si"],
                    help="Rayleigh-Ritz matrix: W^T W (Algorithm 2) or the block-tridiagonal "
                         "T of the block Lanczos recurrence (Section 4.2); or simultaneous "
                         "iteration (Algorithm 1)")
    ap.add_argument("--block-size", type=int, default=0, metavar="P",
                    help="block width p >= k (oversampling, Section 6); 0: p = k")
    ap.add_argument("--time-to-eps", action="store_true",
                    help="dense workloads: for each eps in 1e-1, 1e-2, 1e-3 the smallest q whose "
                         "per-vector error (eq. 3, planted spectrum, measured on the GPU) is at "
                         "most eps, and the time of one solve at that q (each timed form)")
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
    w = workloads.WORKLOADS[args.workload]
    if w.kind == "csr":
        out = run_csr(args, w, bk, torch)
    else:
        out = run_dense(args, w, bk, torch)
    print(json.dumps(out), flush=True)


def base_record(args, w, value, unit, ms, dtype, extra_config):
    cfg = {"workload": f"{args.workload}: {DESCR[args.workload]}",
           "n": w.n, "d": w.d, "k": w.k, "q": w.q, "precision": args.precision,
           "method": args.method, "block_size": args.block_size or w.k,
           "fp32_products": getattr(args, "fp32_products", "limbs")}
    cfg.update(extra_config)
    return {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": cfg,
    }


# ---------------------------------------------------------------- CSR --
def run_csr(args, w, bk, torch):
    dev = torch.device("cuda:0")
    k, q = w.k, w.q
    pw = args.block_size or k
    t_gen = time.perf_counter()
    rp, ci, va = make_csr(w)
    g_rp = torch.from_numpy(rp).to(dev)
    g_ci = torch.from_numpy(ci).to(dev)
    g_va = torch.from_numpy(va).to(dev)
    nnz = int(ci.size)
    bx, by = csr_product_bytes(w.n, w.d, nnz, pw)
    # CSR of A^T: an input layout built once on the GPU (as a caller solving
    # repeatedly would), timed on its own, outside the steps
    tr = bk.csr_transpose(g_rp, g_ci, g_va, w.d)
    torch.cuda.synchronize()
    t0p = time.perf_counter()
    for _ in range(3):
        tr = bk.csr_transpose(g_rp, g_ci, g_va, w.d)
    torch.cuda.synchronize()
    prep_ms = {"csr_transpose": round((time.perf_counter() - t0p) * 1e3 / 3, 4)}
    log(f"inputs ready in {time.perf_counter() - t_gen:.1f}s ({args.workload})")

    def step(timing):
        return bk.svd_csr(g_rp, g_ci, g_va, w.n, w.d, k, q, seed=w.seed_sketch,
                          center=w.center, transpose=tr, timing=timing,
                          method=args.method, block_size=args.block_size,
                          csr_gather=args.csr_gather)

    leg = timed_leg(step, args.steps, args.warmup)
    if args.breakdown:
        log("phase ms/step: " + ", ".join(f"{p}={v:.3f}" for p, v in leg["phases"].items()))
    q_eff = leg["last"].info["q_eff"]
    bytes_per_solve = (q + 1) * (bx + by)
    value = bytes_per_solve / (leg["ms"] * 1e-3) / 1e9
    dom, avg_ms = dominant_product(leg, "csr")
    per_launch = bx if dom == "ax" else by
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    sha = source_sha(["csr.hip"])
    gather = "staged" if args.csr_gather == "staged" else "inplace"
    kernel_key = f"csr_product_{dom}_{args.workload}" + ("_staged" if gather == "staged" else "")
    names = {"ax": "csr_product_kernel (A.X, CSR of A)",
             "aty": "csr_product_kernel (A^T.Y, CSR of A^T)"}
    out = base_record(args, w, value, "GB/s", leg["ms"], "f32",
                      {"product_bytes_per_solve": int(bytes_per_solve), "csr_gather": gather})
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": read_traffic(kernel_key, sha), "kernel": names[dom],
                       "avg_launch_ms": round(avg_ms, 5), "event_steps": leg["n_ev"],
                       "algorithmic_bytes_per_launch": int(per_launch), "source_sha": sha}
    out["phases_ms_per_step"] = {p: round(v, 4) for p, v in leg["phases"].items()}
    out["products_all_kernels"] = products_all_kernels(leg["phases"], q_eff, bx, by)
    out["input_prep_ms_untimed"] = prep_ms
    out["q_eff"] = q_eff
    if args.metrics_q >= 0:
        out["error_measures"] = gpu_error_measures(
            lambda Z, qs: bk.error_metrics_csr(g_rp, g_ci, g_va, w.n, w.d, Z, q_spec=qs,
                                               seed=w.seed_sketch + 1, center=w.center,
                                               transpose=tr),
            leg["last"].Z, args.metrics_q)
    if args.time_to_eps:
        out["time_to_eps"] = {"skipped": "needs the true spectrum (planted dense inputs)"}
    if not (args.no_cpu_baseline and args.no_parity):
        import scipy.sparse as sp
        A = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(w.n, w.d))
        ref, base = oracle_solves(args, w, A, tau=1e-5, f32=True,
                                  seconds=0.0 if args.no_cpu_baseline else args.cpu_seconds)
        if not args.no_cpu_baseline:
            per = base.pop("sec_per_solve")
            base.update({"value": round(bytes_per_solve / per / 1e9, 4), "unit": "GB/s"})
            out["cpu_baseline"] = base
        if not args.no_parity:
            out["parity"] = parity_record(ref, leg["last"], k)
    return out


# -------------------------------------------------------------- dense --
def run_dense(args, w, bk, torch):
    dev = torch.device("cuda:0")
    k, q = w.k, w.q
    pw = args.block_size or k
    compare = args.compare
    if compare == "auto":
        compare = AUTO_COMPARE.get(args.workload, "none") if args.precision == "plain" else "none"
    if args.precision != "plain" or w.dtype == "f64":
        compare = "none"
    t_gen = time.perf_counter()
    sv = workloads.spectrum(w.spectrum, min(w.n, w.d))
    factors = None
    gen_stats = {}
    if args.input == "gaussian":
        args.no_parity = args.no_cpu_baseline = True
        args.time_to_eps = False
        g = torch.Generator(device=dev)
        g.manual_seed(w.seed_matrix)
        A = torch.empty(w.n, w.d, dtype=torch.float32, device=dev)
        for r0 in range(0, w.n, 8192):
            r1 = min(w.n, r0 + 8192)
            A[r0:r1] = torch.randn(r1 - r0, w.d, generator=g, device=dev) / float(np.sqrt(w.d))
    elif w.n * w.d <= 4_000_000:
        A64 = workloads.planted_dense(w.n, w.d, sv, w.seed_matrix, noise=w.noise,
                                      noise_seed=w.seed_noise)
        A = torch.from_numpy(A64).to(dev)
        if w.dtype != "f64":
            A = A.float()
    else:
        # noise-free planted matrices keep their factors for the oracle
        want_f = not args.no_parity and w.noise == 0.0
        res = workloads.planted_dense_torch(w.n, w.d, sv, w.seed_matrix, device=dev,
                                            noise=w.noise, noise_seed=w.seed_noise,
                                            return_factors=want_f, stats=gen_stats)
        A, factors = res if want_f else (res, None)
    if w.dtype == "f64":
        A = A.double()
    prep_ms = {}

    def lowp(prec):
        torch.cuda.synchronize()
        t0p = time.perf_counter()
        if prec == "bf16":
            A_in, kw, a_bytes = bk.quantize(A, "bf16"), {"A_master": A}, 2
            if args.lowp_layout == "both":
                kw["A_t"] = bk.quantize(A, "bf16", transposed=True)
        else:
            A_in, sc = bk.quantize(A, "fp8")
            kw, a_bytes = {"A_master": A, "a_scales": sc}, 1
            if args.lowp_layout == "both":
                kw["A_t"], kw["at_scales"] = bk.quantize(A, "fp8", transposed=True)
        torch.cuda.synchronize()
        prep_ms[f"quantize_{prec}"] = round((time.perf_counter() - t0p) * 1e3, 4)
        return A_in, kw, a_bytes

    x_bytes = 8 if A.dtype == torch.float64 else 4
    main_dtype = "f64" if A.dtype == torch.float64 else "f32"
    if args.precision == "plain":
        A_in, kw, a_bytes = A, {}, A.element_size()
    else:
        A_in, kw, a_bytes = lowp(args.precision)
        main_dtype = args.precision
    torch.cuda.synchronize()
    log(f"inputs ready in {time.perf_counter() - t_gen:.1f}s ({args.workload})")

    def stepper(Ai, kwi):
        def step(timing):
            return bk.svd_dense(Ai, k, q, seed=w.seed_sketch, timing=timing,
                                method=args.method, block_size=args.block_size,
                                fp32_products=args.fp32_products, **kwi)
        return step

    flops_per_product = 2.0 * w.n * w.d * pw
    unit = value_unit("dense", main_dtype, w.n, w.d, pw, a_bytes)

    def leg_summary(leg, dtype, a_b):
        bx, by = dense_product_bytes(w.n, w.d, pw, a_b, x_bytes)
        nprod = 2 * (leg["last"].info["q_eff"] + 1)
        per_solve_bytes = (bx + by) / 2 * nprod
        per_solve_flops = flops_per_product * nprod
        u = value_unit("dense", dtype, w.n, w.d, pw, a_b)
        return {"unit": u, "value": rate(u, per_solve_bytes, per_solve_flops, leg["ms"]),
                "bytes_per_product": (bx + by) / 2, "products_per_solve": nprod,
                "GBps": per_solve_bytes / (leg["ms"] * 1e-3) / 1e9,
                "TFLOPs": per_solve_flops / (leg["ms"] * 1e-3) / 1e12}

    leg = timed_leg(stepper(A_in, kw), args.steps, args.warmup)
    log(f"{main_dtype} leg: {leg['ms']:.2f} ms/solve")
    if args.breakdown:
        log("phase ms/step: " + ", ".join(f"{p}={v:.3f}" for p, v in leg["phases"].items()))
    summ = leg_summary(leg, main_dtype, a_bytes)
    out = base_record(args, w, summ["value"], unit, leg["ms"], main_dtype,
                      {"product_bytes_per_solve": int(summ["bytes_per_product"]
                                                      * summ["products_per_solve"]),
                       "product_flops_per_solve": flops_per_product * summ["products_per_solve"],
                       "input": args.input})
    out["roofline"] = dense_roofline(leg, args, w, main_dtype, a_bytes, x_bytes, pw)
    out["phases_ms_per_step"] = {p: round(v, 4) for p, v in leg["phases"].items()}
    out["q_eff"] = leg["last"].info["q_eff"]
    out["jacobi_sweeps"] = leg["last"].info["jacobi_sweeps"]

    legs = {main_dtype: leg}
    if compare != "none":
        Alp, kwlp, ablp = lowp(compare)
        lp = timed_leg(stepper(Alp, kwlp), args.steps, args.warmup)
        log(f"{compare} leg: {lp['ms']:.2f} ms/solve")
        s2 = leg_summary(lp, compare, ablp)
        out["low_precision"] = {
            "precision": compare, "refine": True, "layout": args.lowp_layout,
            "ms_per_step": round(lp["ms"], 4),
            "speedup_vs_plain": round(leg["ms"] / lp["ms"], 3),
            "products_GBps": round(s2["GBps"], 2), "products_TFLOPs": round(s2["TFLOPs"], 2),
            "roofline": dense_roofline(lp, args, w, compare, ablp, x_bytes, pw),
            "phases_ms_per_step": {p: round(v, 4) for p, v in lp["phases"].items()},
            "q_eff": lp["last"].info["q_eff"]}
        legs[compare] = lp
    out["input_prep_ms_untimed"] = prep_ms
    if gen_stats:
        out["input_storage_rounding_fro"] = gen_stats.get("storage_rounding_fro")

    if args.metrics_q >= 0:
        out["error_measures"] = gpu_error_measures(
            lambda Z, qs: bk.error_metrics_dense(A, Z.to(A.dtype).contiguous(), q_spec=qs,
                                                 seed=w.seed_sketch + 1),
            leg["last"].Z, args.metrics_q)
    if args.time_to_eps:
        tte = {}
        for name, (Ai, kwi) in {main_dtype: (A_in, kw)}.items():
            tte[name] = time_to_eps(lambda qq: bk.svd_dense(Ai, k, qq, seed=w.seed_sketch, **kwi),
                                    lambda Z: per_vector_gpu(bk, A, Z, sv, k, w), q)
        if compare != "none":
            tte[compare] = time_to_eps(
                lambda qq: bk.svd_dense(Alp, k, qq, seed=w.seed_sketch, **kwlp),
                lambda Z: per_vector_gpu(bk, A, Z, sv, k, w), q)
        out["time_to_eps"] = tte

    # the host side: the oracle (float64) for parity, its products for the
    # CPU baseline
    results = {name: lg["last"] for name, lg in legs.items()}
    for lg in legs.values():
        lg["last"] = None
    if compare != "none":
        del Alp, kwlp
    A_host = None
    if not (args.no_parity and args.no_cpu_baseline):
        t_h = time.perf_counter()
        A_host = A.cpu().numpy() if w.n * w.d > 4_000_000 else None
        log(f"A copied to the host in {time.perf_counter() - t_h:.1f}s")
    if not args.no_parity:
        out["parity"] = dense_parity(args, w, k, q, pw, A, A_host, factors, results, torch)
    del factors
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = dense_cpu_baseline(args, w, pw, A, A_host, unit, a_bytes,
                                                 x_bytes, flops_per_product)
    return out


def per_vector_gpu(bk, A, Z, sv, k, w):
    m = bk.error_metrics_dense(A, Z.to(A.dtype).contiguous(), sigma_true=sv[:k + 1], q_spec=0,
                               seed=w.seed_sketch + 1)
    return m.values["per_vector"]


def dense_roofline(leg, args, w, dtype, a_bytes, x_bytes, pw):
    dom, avg_ms = dominant_product(leg, "dense")
    bx, by = dense_product_bytes(w.n, w.d, pw, a_bytes, x_bytes)
    per_launch = bx if dom == "ax" else by
    sha = source_sha(["gemm.hip", "gemm_mfma.hip"])
    kernel_key = f"dense_product_{dom}_{args.workload}_{dtype}"
    names = {"ax": "A.X product (operand pack + product kernel)",
             "aty": "A^T.Y product (operand pack + product kernel + split reduction)"}
    roof = {"bound": "hbm", "achieved": round(per_launch / (avg_ms * 1e-3) / 1e9, 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(per_launch / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": read_traffic(kernel_key, sha), "kernel": names[dom],
            "avg_launch_ms": round(avg_ms, 5), "avg_ms_is": "per product",
            "event_steps": leg["n_ev"], "algorithmic_bytes_per_launch": int(per_launch),
            "source_sha": sha}
    flops = 2.0 * w.n * w.d * pw
    peak, basis = f32_peak(args) if dtype == "f32" else (PEAK_TFS[dtype], None)
    if flops / per_launch > peak * 1e12 / (HBM_PEAK_GBS * 1e9):
        tf = flops / (avg_ms * 1e-3) / 1e12
        roof.update({"bound": "mfma", "achieved": round(tf, 3), "peak": round(peak, 2),
                     "unit": "TFLOP/s", "frac": round(tf / peak, 4),
                     "algorithmic_flops_per_launch": flops})
        if basis:
            roof["peak_basis"] = basis
    return roof


class _DeviceRows:
    """An n x r FP64 device factor read through ``@`` in row blocks copied
    to the host (the product itself runs on the host in float64)."""

    def __init__(self, U, rows=8192):
        self.U, self.rows, self.shape = U, rows, tuple(U.shape)

    def __matmul__(self, X):
        X = np.asarray(X, dtype=np.float64)
        out = np.empty((self.shape[0], X.shape[1]))
        for r0 in range(0, self.shape[0], self.rows):
            r1 = min(self.shape[0], r0 + self.rows)
            out[r0:r1] = self.U[r0:r1].cpu().numpy() @ X
        return out


def dense_parity(args, w, k, q, pw, A, A_host, factors, results, torch):
    """The float64 oracle of the same matrix and the same rounded sketch:
    Algorithm 2 in the coordinates of the planted factors (noise-free
    planted inputs: exact for U diag(sigma) V^T, the FP32 storage of A
    perturbing it by input_storage_rounding_fro), else route A on the
    stored matrix (streamed float64 upcast of the FP32 master)."""
    from oracle import bki, philox

    f64 = w.dtype == "f64"
    tau = 1e-11 if f64 else 1e-5
    Pi = philox.gaussian(w.seed_sketch, w.d, pw)
    if not f64:
        Pi = Pi.astype(np.float32).astype(np.float64)
    if args.method != "bki":
        return {"skipped": "the oracle legs here cover Algorithm 2 with W^T W"}
    t0 = time.perf_counter()
    if factors is not None:
        U, sig, V = factors
        ref = bki.block_krylov_planted(_DeviceRows(U), sig.cpu().numpy(), V.cpu().numpy(), Pi,
                                       k, q, tau=tau, basis=False)
        route = "planted factors (Algorithm 2 on diag(sigma), sketch V^T Pi, Z mapped by U)"
    elif A_host is not None:
        ref = bki.block_krylov(bki.StreamedDense(A_host), Pi, k, q, tau=tau)
        route = "route A on the stored FP32 matrix (float64, streamed row blocks)"
    else:
        Ah = A.cpu().numpy().astype(np.float64)
        ref = bki.block_krylov(Ah, Pi, k, q, tau=tau)
        route = "route A on the stored matrix (float64)"
    out = {"oracle_route": route, "oracle_s": round(time.perf_counter() - t0, 2),
           "oracle_q_eff": int(ref.q_eff)}
    for name, r in results.items():
        out[name] = parity_record(ref, r, k)
    return out


def parity_record(ref, r, k):
    from oracle import metrics
    Zg = r.Z.double().cpu().numpy()
    sg = r.sigma.cpu().numpy()
    rel = float(np.max(np.abs(sg - ref.sigma) / ref.sigma))
    j = 0   # widest leading subspace with relative Ritz gap >= 1e-2
    for jj in range(1, min(k, len(ref.theta) - 1) + 1):
        if (ref.theta[jj - 1] - ref.theta[jj]) / ref.theta[0] >= 1e-2:
            j = jj
    ang = metrics.principal_angle(ref.Z[:, :j], Zg[:, :j]) if j else None
    rel_i = np.abs(sg - ref.sigma) / ref.sigma
    return {"ritz_rel_max": rel, "ritz_rel_median": float(np.median(rel_i)),
            "principal_angle_rad": ang, "gap_separated_j": j,
            "angle_at_k_rad": metrics.principal_angle(ref.Z, Zg),
            "q_eff": int(r.info["q_eff"])}


def oracle_threads():
    from threadpoolctl import threadpool_info
    return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))


def oracle_solves(args, w, A, tau, f32, seconds):
    """Whole oracle solves of the same input (route of --method), repeated
    for about `seconds` (at least one): the last result and the timing."""
    from oracle import bki, philox
    k, q = w.k, w.q
    pw = args.block_size or k
    Pi = philox.gaussian(w.seed_sketch, w.d, pw)
    if f32:
        Pi = Pi.astype(np.float32).astype(np.float64)
    times = []
    ref = None
    t_end = time.perf_counter() + seconds
    while time.perf_counter() < t_end or not times:
        t0 = time.perf_counter()
        if args.method == "si":
            ref = bki.simultaneous_iteration(A, Pi, k, q, center=w.center)
        elif args.method == "lanczos":
            ref = bki.block_lanczos(A, Pi, k, q, center=w.center, tau=tau)[0]
        else:
            ref = bki.block_krylov(A, Pi, k, q, center=w.center, tau=tau)
        times.append(time.perf_counter() - t0)
    threads = oracle_threads()
    per = float(np.median(times))
    base = {"cores": threads, "kind": "oracle",
            "sample": f"{len(times)} whole solves of the same input "
                      f"(median {per * 1e3:.1f} ms/solve, NumPy/SciPy float64; sparse "
                      f"products single-threaded, dense BLAS on {threads} threads)",
            "ms_per_solve": round(per * 1e3, 2), "sec_per_solve": per}
    return ref, base


def dense_cpu_baseline(args, w, pw, A, A_host, unit, a_bytes, x_bytes, flops):
    """The oracle's block products (its float64 operator on the stored
    matrix, as it stands) on the host cores for about --cpu-seconds,
    alternating A.X and A^T.Y, in the unit of the GPU value.  Small inputs
    run whole oracle solves instead."""
    from oracle import bki, philox
    if A_host is None:
        Ah = A.cpu().numpy().astype(np.float64)
        _, base = oracle_solves(args, w, Ah, 1e-11 if w.dtype == "f64" else 1e-5,
                                w.dtype != "f64", args.cpu_seconds)
        per = base.pop("sec_per_solve")
        bx, by = dense_product_bytes(w.n, w.d, pw, a_bytes, x_bytes)
        nprod = 2 * (w.q + 1)
        base.update({"value": round(rate(unit, (bx + by) / 2 * nprod, flops * nprod,
                                         per * 1e3), 6), "unit": unit})
        return base
    op = bki.StreamedDense(A_host)
    X = philox.gaussian(w.seed_sketch, w.d, pw)
    Y = philox.gaussian(w.seed_sketch + 7, w.n, pw)
    times = []
    t_end = time.perf_counter() + args.cpu_seconds
    while time.perf_counter() < t_end or len(times) < 2:
        t0 = time.perf_counter()
        if len(times) % 2 == 0:
            op.mul(X)
        else:
            op.tmul(Y)
        times.append(time.perf_counter() - t0)
    per = float(np.mean(times))
    bx, by = dense_product_bytes(w.n, w.d, pw, a_bytes, x_bytes)
    threads = oracle_threads()
    return {"value": round(rate(unit, (bx + by) / 2, flops, per * 1e3), 6), "unit": unit,
            "cores": threads, "kind": "oracle",
            "sample": f"{len(times)} block products of the full matrix, A.X and A^T.Y "
                      f"alternately, with the oracle's float64 operator on the stored FP32 "
                      f"matrix (StreamedDense, 8192-row blocks upcast, BLAS on {threads} "
                      f"threads); {per * 1e3:.0f} ms per product, a whole oracle solve makes "
                      f"{2 * (w.q + 1)} of them",
            "ms_per_product": round(per * 1e3, 2)}


def gpu_error_measures(fn, Z, qs):
    """eqs. (1)-(3) quantities of the last solve's Z on the GPU (Section 3):
    ||Abar||_F^2, the Frobenius residual (Pythagoras), the spectral residual
    (block Krylov on (I - Z Z^T) Abar, depth qs); no true spectrum here, so
    the ratios are not formed.  Wall time of one call (it synchronizes),
    after a warm-up call."""
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


if __name__ == "__main__":
    main()
