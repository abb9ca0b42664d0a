"""Benchmark of the randomized SVD hot path on one MI355X.

Workload (the dense GPU-resident configuration): A 50000 x 20000 FP32 =
U diag(1/i, i <= 2000) V^T + 1e-4 N(0,1), U and V Haar (seed 2), k = 100,
p = 20, q = 2, 4096 x 4096 block-cyclic tiles, Gaussian test matrix seed 0.
A step is one full randomized SVD (rsvd_factor: Gaussian O, 2q + 2 passes
over A with their orthonormalisations, small SVD, post-processing) with A
already resident in HBM.

Prints one JSON line: value = algorithmic TFLOP/s of the whole
randomized SVD, (2q + 2) * 2 m n l / wall time per step, for the headline
form; per-form wall times, sketch TFLOP/s and sigma errors against the FP64
oracle (timed on the host cores as the cpu_baseline) are included.
"""

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PROFILES = os.path.join(ROOT, "profiles")
PEAK = {"hbm_GBs": 8000.0, "fp32_TF": 157.3, "bf16_TF": 2500.0, "fp8_TF": 5000.0, "fp64_TF": 78.6}
METRIC = "rank-k rSVD wall time & sketch TFLOP/s: BF16-MFMA vs FP32 at matched σ error"
WORKLOAD = dict(name="plain_gpu", m=50000, n=20000, k=100, p=20, q=2, tile=(4096, 4096), seed=0)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel_file, summary):
    """HBM bytes per launch from a committed counter summary, or None when the
    kernel source changed after the counters were taken."""
    import hashlib
    path = os.path.join(PROFILES, summary)
    src = os.path.join(ROOT, "paper_1907_06470_amd", "csrc", kernel_file)
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    fields = {}
    for line in open(path):
        if ":" in line and line.lstrip().startswith("- "):
            key, _, val = line.lstrip()[2:].partition(":")
            fields[key.strip()] = val.strip().strip("`")
    if fields.get("source_sha256") != digest:
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_form(plan, A, steps, warmup):
    ws = plan.workspace(A.device)
    from paper_1907_06470_amd import col_major
    out = (col_major(plan.m, plan.k, device=A.device),
           torch.empty(plan.k, dtype=torch.float64, device=A.device),
           col_major(plan.n, plan.k, device=A.device))
    for _ in range(warmup):
        plan.factor(A, ws=ws, out=out)
    torch.cuda.synchronize()
    # Every fifth timed step (and the last) carries the report: HIP events
    # around each product launch and stage, read after a stream sync.  The
    # other steps run as a caller would, without that instrumentation, which
    # costs about 0.1 ms per call (the sync and ~20 event records).
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        rep = i % 5 == 4 or i == steps - 1
        info = plan.factor(A, ws=ws, out=out, report=rep)[3]
        if rep:
            infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps * 1e3, infos, [o.clone() for o in out]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--forms", default="fp32,bf16,fp8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="dense",
                    choices=["dense", "ooc", "sparse", "hamrle3_like", "circuit5m_like"],
                    help="dense: the headline GPU-resident workload; ooc: A in pinned host "
                         "memory streamed through a 16 GB HBM budget (a separate line)")
    ap.add_argument("--ooc-scale", type=float, default=0.5,
                    help="linear scale of the out-of-core workload (1.0 = 200000 x 100000)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB elementwise copy kernel (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a "
              "design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import workloads
    from paper_1907_06470_amd import Plan

    dev = torch.device("cuda:0")
    if args.workload == "ooc":
        return bench_ooc(args, dev)
    if args.workload == "sparse":
        return bench_sparse(args, dev)
    if args.workload in ("hamrle3_like", "circuit5m_like"):
        return bench_standin(args, dev)
    W = WORKLOAD
    m, n, k, p, q = W["m"], W["n"], W["k"], W["p"], W["q"]
    l = k + p
    t = time.time()
    A, meta = workloads.make(W["name"], device=dev)
    torch.cuda.synchronize()
    log(f"generated A {m}x{n} on the GPU in {time.time() - t:.1f} s")

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst

    flops_pass = 2.0 * m * n * l
    npass = 2 * q + 2
    forms = {}
    for form in args.forms.split(","):
        plan = Plan(m, n, k, p, q, seed=W["seed"], precision=form, tile=W["tile"])
        ms, infos, outs = time_form(plan, A, args.steps, args.warmup)
        # A X launches after the sketch (the power steps): the plain product;
        # the sketch pass of the BF16 form also writes the BF16 copy of A
        nn_ms = np.mean([(i["gemm_nn_ms"] - i["sketch_ms"]) / max(1, i["gemm_nn_launches"] - 1)
                         if i["gemm_nn_launches"] > 1 else i["gemm_nn_ms"] for i in infos])
        sk_ms = np.mean([i["sketch_ms"] for i in infos])
        tn_ms = np.mean([i["gemm_tn_ms"] / max(1, i["gemm_tn_launches"]) for i in infos])
        stage = np.mean([i["stage_ms"] for i in infos], axis=0)
        ebytes = {"fp32": 4, "bf16": 2, "fp8": 1}[form]
        nn_bytes = m * n * ebytes + n * l * ebytes + m * l * 4
        forms[form] = dict(ms_per_step=ms, tflops=npass * flops_pass / (ms * 1e-3) / 1e12,
                           sketch_tflops=flops_pass / (nn_ms * 1e-3) / 1e12,
                           nn_alg_GBs=nn_bytes / (nn_ms * 1e-3) / 1e9,
                           nn_kernel_ms=nn_ms, tn_kernel_ms=tn_ms, sketch_pass_ms=sk_ms,
                           stage_ms=[round(float(x), 4) for x in stage],
                           status=infos[-1]["status"], dropped=infos[-1]["dropped"],
                           jacobi_sweeps=infos[-1]["jacobi_sweeps"], _S=outs[1].cpu().numpy())
        log(f"{form}: {ms:.3f} ms/rSVD, NN kernel {nn_ms:.3f} ms, TN kernel {tn_ms:.3f} ms, "
            f"sketch pass {sk_ms:.3f} ms, "
            f"stages {forms[form]['stage_ms']}")

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import metrics
        from oracle.rsvd import rsvd as oracle_rsvd
        Ah = A.cpu().double().numpy()
        try:
            from threadpoolctl import threadpool_info
            cores = max((x.get("num_threads", 1) for x in threadpool_info()), default=1)
        except Exception:
            cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        ref = oracle_rsvd(Ah, k, p, q, seed=W["seed"])
        t_cpu = time.perf_counter() - t0
        cpu = {"value": npass * flops_pass / t_cpu / 1e12, "unit": "TFLOP/s", "cores": int(cores),
               "kind": "oracle", "seconds": t_cpu,
               "sample": "one full FP64 oracle randomized SVD of the same 50000x20000 A "
                         "(numpy BLAS + Householder QR + one-sided Jacobi)"}
        for f in forms.values():
            f["sigma_err"] = metrics.sigma_err(f["_S"], ref["S"])
        log(f"oracle: {t_cpu:.1f} s on {cores} threads")
    for f in forms.values():
        f.pop("_S", None)

    head_name = "bf16" if "bf16" in forms else next(iter(forms))
    head = forms[head_name]
    if head_name == "fp32":
        roof = {"bound": "mfma", "achieved": round(head["sketch_tflops"], 3),
                "peak": PEAK["fp32_TF"], "unit": "TFLOP/s",
                "frac": round(head["sketch_tflops"] / PEAK["fp32_TF"], 4), "traffic": None,
                "kernel": "k_nn_f32 (sketch / power A*X product)",
                "per_launch": f"2*m*n*l = {flops_pass:.4g} flop"}
    else:
        bpl = m * n * 2 + n * l * 2 + m * l * 4     # A and X in BF16 once, Y in FP32 once
        ach = bpl / (head["nn_kernel_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                "frac": round(ach / PEAK["hbm_GBs"], 4),
                "traffic": measured_traffic("k_gemm_bf16.hip",
                                            "counters_k_nn_bf16_dense_50000x20000.md"),
                "kernel": "k_nn_bf16_dl (A*X product of the power steps, BF16 A streamed "
                          "straight into LDS; the sketch pass is k_nn_bf16_dl_cast reading FP32 A "
                          "and writing the BF16 copy)",
                "per_launch": f"A {m}x{n} bf16 + X {n}x{l} bf16 + Y {m}x{l} fp32 = {bpl} bytes"}
    line = {
        "metric": METRIC, "value": round(head["tflops"], 3), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if head_name == "fp32" else head_name,
        "data": "synthetic",
        "config": {"workload": "dense rSVD 50000x20000 fp32, sigma_i=1/i (i<=2000) + 1e-4 noise, "
                               "k=100 p=20 q=2, 4096x4096 tiles, resident in HBM",
                   "m": m, "n": n, "k": k, "p": p, "q": q, "tile": list(W["tile"]),
                   "parallelism": "single GPU"},
        "forms": {kf: {kk: (float(f"{vv:.6g}") if isinstance(vv, float) else vv)
                       for kk, vv in f.items()} for kf, f in forms.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_sparse(args, dev):
    """Sparse line: CSR 2e6 x 5e5 with 50 Zipf(1.1) columns per row (1e8
    nonzeros), FP32 values; HBM-bound sparse products."""
    import workloads
    from paper_1907_06470_amd import Plan
    m, n, per_row = 2_000_000, 500_000, 50
    k, p, q = 160, 30, 3      # sketch widths above 192 are not implemented (the recipe has l = 330)
    l = k + p
    t = time.time()
    rp, ci, v = workloads.zipf_csr(m, n, per_row, seed=4, device=dev)
    torch.cuda.synchronize()
    nnz = int(ci.numel())
    log(f"generated CSR {m}x{n}, {nnz} nonzeros on the GPU in {time.time() - t:.1f} s")
    plan = Plan(m, n, k, p, q, nnz=nnz)
    ws = plan.workspace(dev)
    for _ in range(args.warmup):
        plan.factor_csr(rp, ci, v, ws=ws)
    torch.cuda.synchronize()
    infos, t0 = [], time.perf_counter()
    for _ in range(args.steps):
        infos.append(plan.factor_csr(rp, ci, v, ws=ws)[3])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    nn_ms = float(np.mean([i["gemm_nn_ms"] / max(1, i["gemm_nn_launches"]) for i in infos]))
    tn_ms = float(np.mean([i["gemm_tn_ms"] / max(1, i["gemm_tn_launches"]) for i in infos]))
    # algorithmic bytes of one A X product: CSR arrays + X once + Y once (FP32)
    alg = nnz * 8 + (m + 1) * 4 + n * l * 4 + m * l * 4
    gbs = alg / (nn_ms * 1e-3) / 1e9
    log(f"sparse: {ms:.2f} ms/rSVD, A X {nn_ms:.3f} ms ({gbs:.0f} GB/s algorithmic), "
        f"A^T Q {tn_ms:.3f} ms, stages {[round(x, 3) for x in infos[-1]['stage_ms']]}")
    line = {
        "metric": "sparse rSVD wall time and A X product GB/s (algorithmic bytes)",
        "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sparse CSR {m}x{n}, {nnz} nonzeros (50 distinct Zipf(1.1) "
                               f"columns per row), k={k} p={p} q={q}",
                   "m": m, "n": n, "nnz": nnz, "k": k, "p": p, "q": q,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_GBs"],
                     "unit": "GB/s", "frac": round(gbs / PEAK["hbm_GBs"], 4), "traffic": None,
                     "kernel": "k_spmm_chunk (A X, CSR)",
                     "per_launch": f"CSR {nnz * 8 + (m + 1) * 4} B + X {n}x{l} fp32 + Y {m}x{l} fp32 = {alg} bytes"},
        "nn_ms": round(nn_ms, 4), "tn_ms": round(tn_ms, 4),
        "stage_ms": [round(float(x), 3) for x in np.mean([i["stage_ms"] for i in infos], axis=0)],
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_standin(args, dev):
    """Sparse COO stand-ins with the shapes of the paper's two SuiteSparse
    test matrices (§4.1; the matrices themselves are absent): banded plus
    uniformly placed entries, int64 coordinates, converted to CSR on the
    device inside every call."""
    import workloads
    from paper_1907_06470_amd import Plan
    r = workloads.SPARSE_STANDINS[args.workload]
    n, nnz = r["n"], r["nnz"]
    k, p, q = 100, 28, 2       # the paper does not state k; l = 128
    l = k + p
    t = time.time()
    ri, ci, v = workloads.banded_random_coo(n, nnz, r["half_width"], r["seed"], device=dev)
    torch.cuda.synchronize()
    log(f"generated COO {n}x{n}, {nnz} entries on the GPU in {time.time() - t:.1f} s")
    plan = Plan(n, n, k, p, q, nnz=nnz, coo=True)
    ws = plan.workspace(dev)
    for _ in range(args.warmup):
        plan.factor_coo(ri, ci, v, ws=ws)
    torch.cuda.synchronize()
    infos, t0 = [], time.perf_counter()
    for _ in range(args.steps):
        infos.append(plan.factor_coo(ri, ci, v, ws=ws)[3])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    nn_ms = float(np.mean([i["gemm_nn_ms"] / max(1, i["gemm_nn_launches"]) for i in infos]))
    tn_ms = float(np.mean([i["gemm_tn_ms"] / max(1, i["gemm_tn_launches"]) for i in infos]))
    alg = nnz * 8 + (n + 1) * 4 + n * l * 4 * 2
    gbs = alg / (nn_ms * 1e-3) / 1e9
    log(f"{args.workload}: {ms:.2f} ms/rSVD, A X {nn_ms:.3f} ms ({gbs:.0f} GB/s algorithmic), "
        f"A^T Q {tn_ms:.3f} ms, stages {[round(x, 3) for x in infos[-1]['stage_ms']]}")
    line = {
        "metric": "sparse rSVD wall time (COO input) and A X product GB/s (algorithmic bytes)",
        "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: COO {n}x{n}, {nnz} entries (band half-width "
                               f"{r['half_width']} plus uniform), int64 indices, k={k} p={p} q={q}",
                   "n": n, "nnz": nnz, "k": k, "p": p, "q": q, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_GBs"],
                     "unit": "GB/s", "frac": round(gbs / PEAK["hbm_GBs"], 4), "traffic": None,
                     "kernel": "k_spmm_chunk (A X, CSR built from the COO input)",
                     "per_launch": f"{alg} bytes"},
        "nn_ms": round(nn_ms, 4), "tn_ms": round(tn_ms, 4),
        "stage_ms": [round(float(x), 3) for x in np.mean([i["stage_ms"] for i in infos], axis=0)],
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_ooc(args, dev):
    """Out-of-core line: A (FP32) in pinned host memory, tiles streamed through
    HBM slots sized by a 16 GB budget; PCIe host-to-device bound."""
    import workloads
    from paper_1907_06470_amd import Plan
    r = workloads.RECIPES["ooc"]
    sc = args.ooc_scale
    m, n = int(round(r["m"] * sc)), int(round(r["n"] * sc))
    # sketch widths above 192 are not implemented: keep l = 190 (k = 160, p = 30)
    k, p, q = 160, 30, r["q"]
    budget = 16 * 10 ** 9
    t = time.time()
    Ad, _ = workloads.make("ooc", device=dev, scale=sc)
    Ah = torch.empty((m, n), dtype=torch.float32, pin_memory=True)
    Ah.copy_(Ad)
    del Ad
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"generated A {m}x{n} ({m * n * 4 / 1e9:.1f} GB) into pinned host memory in "
        f"{time.time() - t:.1f} s")
    # pinned host -> device peak of this machine (one 2 GiB copy, best of 3)
    src = Ah.view(-1)[: 1 << 29]
    dst = torch.empty(src.shape, dtype=src.dtype, device=dev)
    peak = 0.0
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        peak = max(peak, src.numel() * 4 / (time.perf_counter() - t0) / 1e9)
    del dst
    plan = Plan(m, n, k, p, q, tile=r["tile"], host=True, hbm_budget=budget)
    ws = plan.workspace(dev)
    for _ in range(args.warmup):
        plan.factor(Ah, ws=ws)
    torch.cuda.synchronize()
    infos, t0 = [], time.perf_counter()
    for _ in range(args.steps):
        infos.append(plan.factor(Ah, ws=ws)[3])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    h2d = float(np.mean([i["h2d_bytes"] for i in infos]))
    gbs = h2d / (ms * 1e-3) / 1e9
    log(f"ooc: {ms:.1f} ms/rSVD, {h2d / 1e9:.1f} GB host->device per rSVD, {gbs:.1f} GB/s, "
        f"pinned peak {peak:.1f} GB/s, {infos[-1]['slots']} slots, {infos[-1]['tile_loads']} loads")
    line = {
        "metric": "out-of-core rSVD: host-to-device GB/s over the whole factorisation",
        "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"out-of-core dense rSVD {m}x{n} fp32 in pinned host memory, "
                               f"sigma_i=i^-0.8 (i<=500) + 1e-5 noise, k={k} p={p} q={q}, "
                               f"8192x8192 tiles, HBM budget 16 GB",
                   "m": m, "n": n, "k": k, "p": p, "q": q, "parallelism": "single GPU"},
        "roofline": {"bound": "pcie", "achieved": round(gbs, 2), "peak": round(peak, 2),
                     "unit": "GB/s", "frac": round(gbs / peak, 4), "traffic": None,
                     "peak_kind": "measured pinned host-to-device copy of 2 GiB"},
        "h2d_bytes_per_step": h2d, "slots": infos[-1]["slots"],
        "tile_loads": infos[-1]["tile_loads"], "ws_bytes": infos[-1]["ws_bytes"],
        "stage_ms": [round(float(x), 2) for x in np.mean([i["stage_ms"] for i in infos], axis=0)],
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
