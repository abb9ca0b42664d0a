"""Benchmark of the randomized SVD hot path on one MI355X.

Default workload (the dense GPU-resident configuration the headline metric is
quoted on): A 50000 x 20000 FP32 = U diag(1/i, i <= 2000) V^T + 1e-4 N(0,1),
U and V Haar (seed 2), k = 100, p = 20, q = 2, 4096 x 4096 block-cyclic
tiles, Gaussian test matrix seed 0.  A step is one full randomized SVD
(rsvd_factor: Gaussian O, 2q + 2 passes over A with their
orthonormalisations, small SVD, post-processing) with A already resident in
HBM.

Prints one JSON line: value = algorithmic TFLOP/s of the whole randomized
SVD, (2q + 2) * 2 m n l / wall time per step, for the headline (BF16) form.
Every form (FP32, BF16, FP8) also reports its wall time (the mean over the
timed steps and the median of 5 single synchronised runs), the sketch-pass
TFLOP/s (2 m n l over the Y = A O launch), the product kernels' achieved
bandwidth from HIP events around every launch, and its accuracy against the
FP64 oracle run on the same A: sigma error, subspace angles of U and V, the
relative difference of the residual ||A - U S V^T||_F and the orthogonality
of U and V.  The oracle's run is timed on the host cores as the cpu_baseline.

Other lines (--workload): mixed (65536 x 32768, k = 128, p = 32, q = 3, the
three forms plus the adjoint), sparse (CSR 2e6 x 5e5, l = 330), ooc (A in
pinned host memory under a 16 GB HBM budget, l = 230) and the two COO
stand-ins.
"""

import argparse
import json
import os
import platform
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
EBYTES = {"fp32": 4, "bf16": 2, "fp8": 1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel_files, summary):
    """HBM bytes per launch from a committed counter summary, or None when a
    source the traffic depends on changed after the counters were taken (the
    summary's source_sha256 is the SHA-256 of those files, concatenated in the
    order given)."""
    import hashlib
    if isinstance(kernel_files, str):
        kernel_files = (kernel_files,)
    path = os.path.join(PROFILES, summary)
    srcs = [os.path.join(ROOT, "paper_1907_06470_amd", "csrc", f) for f in kernel_files]
    if not (os.path.exists(path) and all(os.path.exists(f) for f in srcs)):
        return None
    digest = hashlib.sha256(b"".join(open(f, "rb").read() for f in srcs)).hexdigest()
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


def host_facts():
    """What the CPU baseline ran on: model, BLAS, threads."""
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas, threads = "unknown", None
    try:
        from threadpoolctl import threadpool_info
        for x in threadpool_info():
            if x.get("user_api") == "blas":
                blas = f"{x.get('internal_api')} {x.get('version')}"
                threads = int(x.get("num_threads", 1))
                break
    except Exception:
        pass
    aff = len(os.sched_getaffinity(0))
    return {"cpu_model": model, "blas": blas, "blas_threads": threads or aff,
            "affinity_cpus": aff, "os_cpu_count": os.cpu_count()}


def time_steps(run, steps, warmup, report_every=5):
    """Mean wall time per step over `steps` back-to-back calls, plus the
    reports of every report_every-th call (and the last)."""
    for _ in range(warmup):
        run(False)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        rep = i % report_every == report_every - 1 or i == steps - 1
        info = run(rep)
        if rep:
            infos.append(info)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, infos


def median_runs(run, count=5):
    """Median of `count` single runs, each synchronised on both sides."""
    ts = []
    for _ in range(count):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(False)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def kernel_rows(form, m, n, l, lp, infos):
    """Per-launch device time (HIP events recorded on the launch stream) and
    algorithmic work of the three product kernels of one form."""
    eb = EBYTES[form]
    fused = form == "bf16" and lp == 128     # the BF16 sketch pass also writes the BF16 copy
    sk_ms = float(np.mean([i["sketch_ms"] for i in infos]))
    nn_launch = infos[-1]["gemm_nn_launches"]
    tn_launch = infos[-1]["gemm_tn_launches"]
    nn_ms = float(np.mean([(i["gemm_nn_ms"] - i["sketch_ms"]) / max(1, i["gemm_nn_launches"] - 1)
                           for i in infos])) if nn_launch > 1 else None
    tn_ms = float(np.mean([i["gemm_tn_ms"] / max(1, i["gemm_tn_launches"]) for i in infos]))
    flops = 2.0 * m * n * l
    nn_bytes = m * n * eb + n * l * eb + m * l * 4
    tn_bytes = m * n * eb + m * l * eb + n * l * 4
    sk_bytes = (m * n * 4 + m * n * 2 + n * l * 2 + m * l * 4) if fused else nn_bytes
    names = {"fp32": ("k_nn_f32", "k_nn_f32", "k_tn_f32"),
             "bf16": ("k_nn_bf16_dl_cast" if fused else
                      "k_nn_bf16_dl" if lp in (128, 160) else "k_nn_bf16",
                      "k_nn_bf16_dl" if lp in (128, 160) else "k_nn_bf16",
                      "k_tn_bf16_dl" if lp in (128, 160) else "k_tn_bf16"),
             "fp8": ("k_nn_fp8_dl" if lp in (128, 160) else "k_nn_fp8",) * 2 +
                    ("k_nn_fp8_dl on the transposed copy" if lp in (128, 160)
                     else "k_nn_fp8 on the transposed copy",)}[form]
    rows = [dict(role="sketch Y = A O", kernel=names[0], launches=1, ms=sk_ms, bytes=sk_bytes,
                 flops=flops)]
    if nn_ms is not None:
        rows.append(dict(role="power A X", kernel=names[1], launches=nn_launch - 1, ms=nn_ms,
                         bytes=nn_bytes, flops=flops))
    rows.append(dict(role="A^T Q (power and projection)", kernel=names[2], launches=tn_launch,
                     ms=tn_ms, bytes=tn_bytes, flops=flops))
    for r in rows:
        r["GBs"] = r["bytes"] / (r["ms"] * 1e-3) / 1e9
        r["TFs"] = r["flops"] / (r["ms"] * 1e-3) / 1e12
        r["total_ms"] = r["ms"] * r["launches"]
    return rows


def roofline_of(form, rows, traffic_files, m, n, l):
    """Roofline object of the kernel with the most device time per rSVD."""
    dom = max(rows, key=lambda r: r["total_ms"])
    if form == "fp32":
        roof = {"bound": "mfma", "achieved": round(dom["TFs"], 3), "peak": PEAK["fp32_TF"],
                "unit": "TFLOP/s", "frac": round(dom["TFs"] / PEAK["fp32_TF"], 4),
                "traffic": None, "per_launch": f"2*m*n*l = {dom['flops']:.4g} flop"}
    else:
        tr = None
        spec = traffic_files.get(dom["kernel"])
        if spec:
            tr = measured_traffic(*spec)
        roof = {"bound": "hbm", "achieved": round(dom["GBs"], 1), "peak": PEAK["hbm_GBs"],
                "unit": "GB/s", "frac": round(dom["GBs"] / PEAK["hbm_GBs"], 4), "traffic": tr,
                "per_launch": f"{dom['bytes']} algorithmic bytes ({form} A {m}x{n}, panel "
                              f"{l} columns, FP32 output)"}
    roof.update(kernel=dom["kernel"], role=dom["role"], launch_ms=round(dom["ms"], 5),
                launches_per_step=dom["launches"])
    return roof


def accuracy(A_dev, plan, out, ref, r_ref):
    """sigma error, subspace angles, residual and orthogonality of one form
    against the oracle (R13 metrics)."""
    from oracle import metrics
    U, S, V = out
    r_hat = float(plan.residual(A_dev, U, S, V).item())
    Un, Sn, Vn = U.cpu().double().numpy(), S.cpu().numpy(), V.cpu().double().numpy()
    return {"sigma_err": metrics.sigma_err(Sn, ref["S"]),
            "sin_u": metrics.sin_theta(ref["U"], Un), "sin_v": metrics.sin_theta(ref["V"], Vn),
            "resid": r_hat, "resid_rel": abs(r_hat - r_ref) / r_ref,
            "orth_u": metrics.orth_err(Un), "orth_v": metrics.orth_err(Vn)}


def run_oracle(Ah, k, p, q, seed):
    from oracle import metrics
    from oracle.rsvd import rsvd as oracle_rsvd
    times = {}
    t0 = time.perf_counter()
    ref = oracle_rsvd(Ah, k, p, q, seed=seed, times=times)
    t_cpu = time.perf_counter() - t0
    r_ref = metrics.residual_fro(Ah, ref["U"], ref["S"], ref["V"])
    return ref, r_ref, t_cpu, times


def fmt(d):
    return {kk: (float(f"{vv:.6g}") if isinstance(vv, float) else vv) for kk, vv in d.items()}


def copy_calibration(dev):
    """One plain elementwise copy kernel of known size (reads 1 GiB, writes
    1 GiB): the reference that scales the HBM byte counters."""
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


def bench_dense(args, dev, recipe):
    """The headline line (recipe plain_gpu) or the mixed-precision line
    (recipe mixed, with the adjoint)."""
    import workloads
    from paper_1907_06470_amd import Plan, col_major
    r = workloads.RECIPES[recipe]
    m, n, k, p, q = r["m"], r["n"], r["k"], r["p"], r["q"]
    l, seed, tile = k + p, 0, r["tile"]
    lp = -(-l // 32) * 32
    t = time.time()
    A, meta = workloads.make(recipe, device=dev)
    torch.cuda.synchronize()
    log(f"generated A {m}x{n} on the GPU in {time.time() - t:.1f} s")
    if args.copy_calibration:
        copy_calibration(dev)
    flops_pass = 2.0 * m * n * l
    npass = 2 * q + 2
    forms, outs = {}, {}
    for form in args.forms.split(","):
        plan = Plan(m, n, k, p, q, seed=seed, precision=form, tile=tile)
        ws = plan.workspace(dev)
        out = (col_major(m, k, device=dev), torch.empty(k, dtype=torch.float64, device=dev),
               col_major(n, k, device=dev))

        def run(rep, plan=plan, ws=ws, out=out):
            return plan.factor(A, ws=ws, out=out, report=rep)[3]

        ms, infos = time_steps(run, args.steps, args.warmup)
        med = median_runs(run)
        rows = kernel_rows(form, m, n, l, lp, infos)
        stage = np.mean([i["stage_ms"] for i in infos], axis=0)
        sk = rows[0]
        forms[form] = dict(ms_per_step=ms, ms_median5=med,
                           tflops=npass * flops_pass / (ms * 1e-3) / 1e12,
                           sketch_pass_ms=sk["ms"], sketch_tflops=sk["TFs"],
                           kernels=[fmt({kk: vv for kk, vv in rr.items()}) for rr in rows],
                           stage_ms=[round(float(x), 4) for x in stage],
                           status=infos[-1]["status"], dropped=infos[-1]["dropped"],
                           jacobi_sweeps=infos[-1]["jacobi_sweeps"])
        forms[form]["_rows"] = rows
        outs[form] = (plan, tuple(o.clone() for o in out))
        log(f"{form}: {ms:.3f} ms/rSVD (median of 5: {med:.3f}), sketch pass {sk['ms']:.3f} ms "
            f"({sk['TFs']:.1f} TFLOP/s), kernels " +
            ", ".join(f"{rr['kernel']} {rr['ms']:.3f} ms x{rr['launches']}" for rr in rows))

    bwd = None
    if recipe == "mixed" and not args.no_backward:
        bwd = bench_backward(A, m, n, k, p, q, seed, tile, dev, args)

    cpu = None
    if not args.no_cpu_baseline:
        Ah = A.cpu().double().numpy()
        facts = host_facts()
        ref, r_ref, t_cpu, times = run_oracle(Ah, k, p, q, seed)
        cpu = {"value": npass * flops_pass / t_cpu / 1e12, "unit": "TFLOP/s",
               "cores": facts["blas_threads"], "kind": "oracle", "seconds": t_cpu,
               "sample": f"one full FP64 oracle randomized SVD of the same {m}x{n} A "
                         "(numpy BLAS products + Householder QR + one-sided Jacobi)",
               "stage_s": {kk: round(vv, 3) for kk, vv in times.items()}, **facts}
        for form, (plan, out) in outs.items():
            forms[form].update(accuracy(A, plan, out, ref, r_ref))
        log(f"oracle: {t_cpu:.1f} s on {facts['blas_threads']} threads ({facts['blas']}); "
            f"stages {cpu['stage_s']}")
        if bwd is not None:
            bwd.update(closed_form_check(A, Ah, bwd.pop("_factors"), bwd.pop("_gA"), bwd.pop("_w")))
        del Ah
    if bwd is not None:
        for key in ("_factors", "_gA", "_w"):
            bwd.pop(key, None)

    head_name = "bf16" if "bf16" in forms else next(iter(forms))
    head = forms[head_name]
    ptag = f"{recipe}_{m}x{n}"
    traffic_files = {kern: ("k_gemm_bf16.hip", f"counters_{kern}_{ptag}.md")
                     for kern in ("k_nn_bf16_dl", "k_tn_bf16_dl", "k_nn_bf16_dl_cast", "k_nn_bf16",
                                  "k_tn_bf16")}
    traffic_files.update({kern: ("k_gemm_fp8.hip", f"counters_k_nn_fp8_{ptag}.md")
                          for kern in ("k_nn_fp8_dl", "k_nn_fp8")})
    roof = roofline_of(head_name, head["_rows"], traffic_files, m, n, l)
    for f in forms.values():
        f.pop("_rows", None)
    spec = r["spectrum"]
    line = {
        "metric": METRIC, "value": round(head["tflops"], 3), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if head_name == "fp32" else head_name,
        "data": "synthetic",
        "config": {"workload": f"dense rSVD {m}x{n} fp32, sigma_i=i^-{spec[2]:g} "
                               f"(i<={spec[1]}) + {r['noise']:g} noise, k={k} p={p} q={q}, "
                               f"{tile[0]}x{tile[1]} tiles, resident in HBM",
                   "m": m, "n": n, "k": k, "p": p, "q": q, "tile": list(tile),
                   "parallelism": "single GPU"},
        "forms": {kf: fmt(f) for kf, f in forms.items()},
        "roofline": roof,
        "cpu_baseline": fmt(cpu) if cpu else None,
    }
    if bwd is not None:
        line["backward"] = fmt(bwd)
    if recipe != "plain_gpu":
        line["metric"] = ("mixed-precision rSVD wall time per form (FP32, BF16, FP8) with "
                          "accuracy against the FP64 oracle, and the adjoint")
    print(json.dumps(line), flush=True)


def bench_backward(A, m, n, k, p, q, seed, tile, dev, args):
    """The adjoint after a forward pass in the form args.bwd_form: loss
    L = sum w_i s_i + ||A - U S V^T||_F^2 (w_i ~ U(0,1), seed 7), its
    cotangents from torch autograd on the factors, then rsvd_backward timed
    with HIP events on the stream it runs on."""
    from paper_1907_06470_amd import Plan
    form = args.bwd_form
    plan = Plan(m, n, k, p, q, seed=seed, precision=form, tile=tile, backward=True)
    ws = plan.workspace(dev)
    U, S, V, _ = plan.factor(A, ws=ws)
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    w = torch.rand(k, generator=g, device=dev, dtype=torch.float64)
    Ut = U.detach().clone().requires_grad_(True)
    St = S.detach().clone().requires_grad_(True)
    Vt = V.detach().clone().requires_grad_(True)
    R = A.double() - (Ut.double() * St) @ Vt.double().T
    loss = (w * St).sum() + (R * R).sum()
    gU, gS, gV = torch.autograd.grad(loss, (Ut, St, Vt))
    del R
    torch.cuda.empty_cache()
    gU, gV = gU.float(), gV.float()
    for _ in range(args.warmup):
        plan.backward(A, gU, gS, gV, ws=ws, report=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    gA = None
    for _ in range(max(1, min(args.steps, 5))):
        torch.cuda.synchronize()
        e0.record()
        gA, _ = plan.backward(A, gU, gS, gV, ws=ws, report=False)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    lp, kp = -(-(k + p) // 32) * 32, -(-k // 32) * 32
    outer_flops = 2.0 * m * n * (lp + 2 * kp)      # gA = [U_l | P2 | P3] [R1 | V_k | R3]^T
    log(f"backward ({form} forward recomputed): {ms:.2f} ms; the gA outer product is "
        f"{outer_flops:.3g} flop and {m * n * 4 / 1e9:.2f} GB written")
    return {"form": form, "ms_median": ms, "gA_bytes": m * n * 4, "outer_flops": outer_flops,
            "_factors": (U, S, V), "_gA": gA, "_w": w}


def closed_form_check(A, Ah, factors, gA, w, rows=256):
    """The gradient of the loss above is the direct term 2 (A - U S V^T) plus
    the adjoint's gA; for rSVD factors (U^T A = S V^T) the sum is exactly
    U diag(w) V^T + 2 A (I - V V^T).  Checked on a seeded sample of rows in
    FP64 on the host."""
    U, S, V = (x.cpu().double().numpy() for x in factors)
    wn = w.cpu().numpy()
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(Ah.shape[0], size=min(rows, Ah.shape[0]), replace=False))
    Ar = Ah[idx]
    ref = (U[idx] * wn) @ V.T + 2.0 * (Ar - (Ar @ V) @ V.T)
    got = gA[torch.as_tensor(idx, device=gA.device)].cpu().double().numpy()
    got = got + 2.0 * (Ar - (U[idx] * S) @ V.T)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    log(f"backward closed form on {len(idx)} rows: relative error {err:.2e}")
    return {"closed_form_rel_err": err, "closed_form_rows": int(len(idx))}


def bench_sparse(args, dev):
    """Sparse line: CSR 2e6 x 5e5 with 50 Zipf(1.1) columns per row (1e8
    nonzeros), FP32 values, k = 300, p = 30, q = 3; HBM-bound sparse
    products.  Accuracy at this size is checked by properties that hold for
    any randomized SVD: orthonormal U and V, and U^T A = S V^T on a seeded
    sample of columns."""
    import workloads
    from paper_1907_06470_amd import Plan
    m, n, per_row = 2_000_000, 500_000, 50
    k, p, q = args.sparse_k, 30, 3
    l = k + p
    t = time.time()
    rp, ci, v = workloads.zipf_csr(m, n, per_row, seed=4, device=dev)
    torch.cuda.synchronize()
    nnz = int(ci.numel())
    log(f"generated CSR {m}x{n}, {nnz} nonzeros on the GPU in {time.time() - t:.1f} s")
    if args.copy_calibration:
        copy_calibration(dev)
    plan = Plan(m, n, k, p, q, nnz=nnz)
    ws = plan.workspace(dev)

    def run(rep):
        return plan.factor_csr(rp, ci, v, ws=ws, report=rep)[3]

    ms, infos = time_steps(run, args.steps, args.warmup, report_every=1)
    U, S, V, _ = plan.factor_csr(rp, ci, v, ws=ws)
    nn_ms = float(np.mean([i["gemm_nn_ms"] / max(1, i["gemm_nn_launches"]) for i in infos]))
    tn_ms = float(np.mean([i["gemm_tn_ms"] / max(1, i["gemm_tn_launches"]) for i in infos]))
    # algorithmic bytes of one product: compressed arrays + X once + Y once (FP32)
    nn_alg = nnz * 8 + (m + 1) * 4 + n * l * 4 + m * l * 4
    tn_alg = nnz * 8 + (n + 1) * 4 + m * l * 4 + n * l * 4
    nn_gbs, tn_gbs = nn_alg / (nn_ms * 1e-3) / 1e9, tn_alg / (tn_ms * 1e-3) / 1e9
    nn_tot = nn_ms * infos[-1]["gemm_nn_launches"]
    tn_tot = tn_ms * infos[-1]["gemm_tn_launches"]
    dom = ("A^T Q (CSC copy)", tn_ms, tn_alg, tn_gbs) if tn_tot >= nn_tot else \
          ("A X (CSR)", nn_ms, nn_alg, nn_gbs)
    # properties: orthonormal factors, U^T A = S V^T on sampled columns
    from oracle import metrics
    import scipy.sparse as sps
    M = sps.csr_matrix((v.cpu().numpy().astype(np.float64), ci.cpu().numpy(), rp.cpu().numpy()),
                       shape=(m, n))
    Un, Sn, Vn = U.cpu().double().numpy(), S.cpu().numpy(), V.cpu().double().numpy()
    cols = np.sort(np.random.default_rng(5).choice(n, size=2048, replace=False))
    lhs = (M[:, cols].T @ Un).T
    rel = float(np.max(np.abs(lhs - Sn[:, None] * Vn[cols].T)) / Sn[0])
    props = {"orth_u": metrics.orth_err(Un), "orth_v": metrics.orth_err(Vn),
             "UtA_minus_SVt_rel_sampled": rel, "sampled_columns": 2048}
    log(f"sparse: {ms:.2f} ms/rSVD, A X {nn_ms:.3f} ms ({nn_gbs:.0f} GB/s algorithmic), "
        f"A^T Q {tn_ms:.3f} ms ({tn_gbs:.0f} GB/s), stages "
        f"{[round(x, 3) for x in infos[-1]['stage_ms']]}, properties {props}")
    # measured HBM traffic of one A^T Q product (committed counter summary)
    traffic = measured_traffic(("k_sparse.hip", "plan.cpp", "plan.h"),
                               f"counters_k_spmm_chunk_sparse_{m}x{n}.md") \
        if dom[0].startswith("A^T Q") and l == 330 else None
    cpu = None
    if not args.no_cpu_baseline:
        # bounded sample: the oracle's FP64 product A O on the first tenth of
        # the rows (scipy CSR x dense), scaled to the 8 passes over A of one
        # rSVD (products only: a lower bound of the oracle's time).  The panel
        # comes from numpy's generator: the product's cost does not depend on
        # its values, and the oracle's own Philox panel alone takes ~30 s here.
        rows = m // 10
        O = np.random.default_rng(0).standard_normal((n, l))
        t0 = time.perf_counter()
        _ = M[:rows] @ O
        t_s = time.perf_counter() - t0
        facts = host_facts()
        cpu = {"value": round(t_s * 10 * 8 * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
               "seconds": round(t_s, 3),
               "sample": f"FP64 CSR x dense product of rows 0..{rows} (1/10 of A) with an "
                         f"{n}x{l} Gaussian panel (scipy, one thread), scaled x10 x8 passes: "
                         "the oracle's products alone, a lower bound of its rSVD time",
               **{kk: facts[kk] for kk in ("cpu_model", "affinity_cpus") if kk in facts}}
        log(f"oracle sample: {t_s:.2f} s for 1/10 of one product")
    line = {
        "metric": "sparse rSVD wall time and sparse-product GB/s (algorithmic bytes)",
        "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sparse CSR {m}x{n}, {nnz} nonzeros (50 distinct Zipf(1.1) "
                               f"columns per row), k={k} p={p} q={q}",
                   "m": m, "n": n, "nnz": nnz, "k": k, "p": p, "q": q,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(dom[3], 1), "peak": PEAK["hbm_GBs"],
                     "unit": "GB/s", "frac": round(dom[3] / PEAK["hbm_GBs"], 4),
                     "traffic": traffic,
                     "traffic_GBs": round(traffic / (dom[1] * 1e-3) / 1e9, 1) if traffic else None,
                     "kernel": f"sparse product {dom[0]}: for every column slice the layout "
                               "change, the chunk products and carries, and (A^T Q) the head "
                               "columns' LDS blocks and their block sums",
                     "launch_ms": round(dom[1], 4),
                     "per_launch": f"compressed arrays + X once + Y once (FP32) = {dom[2]} bytes; "
                                   "traffic: measured bytes of the same product (row gathers)"},
        "nn_ms": round(nn_ms, 4), "tn_ms": round(tn_ms, 4), "nn_GBs": round(nn_gbs, 1),
        "tn_GBs": round(tn_gbs, 1),
        "stage_ms": [round(float(x), 3) for x in np.mean([i["stage_ms"] for i in infos], axis=0)],
        "jacobi_sweeps": infos[-1]["jacobi_sweeps"], "properties": fmt(props),
        "cpu_baseline": cpu,
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

    def run(rep):
        return plan.factor_coo(ri, ci, v, ws=ws, report=rep)[3]

    ms, infos = time_steps(run, args.steps, args.warmup, report_every=1)
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
                     "kernel": "sparse product A X (CSR built from the COO input)",
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
    k, p, q = r["k"], r["p"], r["q"]
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

    def run(rep):
        return plan.factor(Ah, ws=ws, report=rep)[3]

    ms, infos = time_steps(run, args.steps, args.warmup, report_every=1)
    h2d = float(np.mean([i["h2d_bytes"] for i in infos]))
    gbs = h2d / (ms * 1e-3) / 1e9
    log(f"ooc: {ms:.1f} ms/rSVD, {h2d / 1e9:.1f} GB host->device per rSVD, {gbs:.1f} GB/s, "
        f"pinned peak {peak:.1f} GB/s, {infos[-1]['slots']} slots, {infos[-1]['tile_loads']} loads")
    acc = None
    if args.accuracy:
        U, S, V, _ = plan.factor(Ah, ws=ws)
        Ahd = Ah.numpy().astype(np.float64)
        ref, r_ref, t_cpu, _ = run_oracle(Ahd, k, p, q, 0)
        from oracle import metrics
        Un, Sn, Vn = U.cpu().double().numpy(), S.cpu().numpy(), V.cpu().double().numpy()
        acc = {"sigma_err": metrics.sigma_err(Sn, ref["S"]),
               "sin_u": metrics.sin_theta(ref["U"], Un), "sin_v": metrics.sin_theta(ref["V"], Vn),
               "resid_rel": abs(metrics.residual_fro(Ahd, Un, Sn, Vn) - r_ref) / r_ref,
               "orth_u": metrics.orth_err(Un), "orth_v": metrics.orth_err(Vn),
               "oracle_s": t_cpu}
        log(f"ooc accuracy: {acc}")
    line = {
        "metric": "out-of-core rSVD: host-to-device GB/s over the whole factorisation",
        "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"out-of-core dense rSVD {m}x{n} fp32 in pinned host memory, "
                               f"sigma_i=i^-0.8 (i<={int(round(500 * sc))}) + 1e-5 noise, "
                               f"k={k} p={p} q={q}, 8192x8192 tiles, HBM budget 16 GB",
                   "m": m, "n": n, "k": k, "p": p, "q": q, "scale": sc,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "pcie", "achieved": round(gbs, 2), "peak": round(peak, 2),
                     "unit": "GB/s", "frac": round(gbs / peak, 4), "traffic": None,
                     "peak_kind": "measured pinned host-to-device copy of 2 GiB"},
        "h2d_bytes_per_step": h2d, "slots": infos[-1]["slots"],
        "tile_loads": infos[-1]["tile_loads"], "ws_bytes": infos[-1]["ws_bytes"],
        "stage_ms": [round(float(x), 2) for x in np.mean([i["stage_ms"] for i in infos], axis=0)],
        "accuracy": fmt(acc) if acc else None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--forms", default="fp32,bf16,fp8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="dense",
                    choices=["dense", "mixed", "ooc", "sparse", "hamrle3_like", "circuit5m_like"],
                    help="dense: the headline GPU-resident workload; the others are separate "
                         "lines")
    ap.add_argument("--ooc-scale", type=float, default=0.5,
                    help="linear scale of the out-of-core workload (1.0 = 200000 x 100000)")
    ap.add_argument("--accuracy", action="store_true",
                    help="ooc: also run the FP64 oracle on the same A")
    ap.add_argument("--sparse-k", type=int, default=300)
    ap.add_argument("--no-backward", action="store_true", help="mixed: skip the adjoint")
    ap.add_argument("--bwd-form", default="bf16", help="mixed: form of the forward the adjoint recomputes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB elementwise copy kernel (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a "
              "design, not part of this build", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.workload == "ooc":
        return bench_ooc(args, dev)
    if args.workload == "sparse":
        return bench_sparse(args, dev)
    if args.workload in ("hamrle3_like", "circuit5m_like"):
        return bench_standin(args, dev)
    return bench_dense(args, dev, "plain_gpu" if args.workload == "dense" else "mixed")


if __name__ == "__main__":
    main()
