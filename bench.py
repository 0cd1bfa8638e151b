"""Benchmark: hyper-systolic product forward + backward at n = 8192 on one GPU.

One step = the whole hot path over one batch of synthetic input:
C = A . B, dA = G . B^T, dB = A^T . G (three products on the schedule
(p, K)), each with its operand preparation, main MFMA loop and back-shift.
Inputs: A, B ~ N(0, 1) rows scaled log-uniformly in [1e-3, 1e3],
G ~ N(0, 1), seeded, resident in HBM before the timed region.

Prints ONE JSON line.  ``value`` is the useful TFLOP/s of the split-BF16
form (3 * 2 n^3 flops per step over the timed wall clock); the plain FP32
form of the same step is measured beside it under ``comparison``.
``accuracy`` holds, for both forms, the errors of the last timed step's C,
dA and dB against the FP64 oracle rows that the CPU baseline computes.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "bf16": 2516.6, "f16": 2516.6, "fp8": 5033.2, "f32": 157.3, "f64": 78.6, "hbm_gbs": 8000.0,
}
# The published FP32 vector peak (256 CUs x 256 flops per clock x 2.4 GHz)
# is the ALU roofline of the n-body kernel.  It counts two FMAs per lane and
# clock; plain (unpacked) FMAs measured 74.9 TFLOP/s on the chip, and every
# kernel here leaves packed FP32 instructions out.
VALU_F32_PEAK = PEAK["f32"]
# flops of one body-body interaction: 3 differences, 3 FMAs for the squared
# distance plus softening, 1 reciprocal square root, 4 products / differences
# for the potential and the factor m / s^(3/2), 3 FMAs into the acceleration
NBODY_FLOPS = 20
MFMA_PRODUCTS = {"split3_bf16": 6, "bf16": 1, "f16": 1, "f32": 1, "f64": 1, "fp8_e4m3": 1, "fp8_e4m3_r1": 3,
                 "split2_f16": 3}
MFMA_PEAK_KEY = {"split3_bf16": "bf16", "bf16": "bf16", "f16": "f16", "f32": "f32", "f64": "f64",
                 "fp8_e4m3": "fp8", "fp8_e4m3_r1": "fp8", "split2_f16": "f16"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (10; 200 for gemv, whose steps are 40 us launches replayed from a graph)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192, help="square size (default workload)")
    ap.add_argument("--shape", default="",
                    help="M,Kd,N for a rectangular workload, e.g. 16384,8192,16384 (overrides --n)")
    ap.add_argument("--inputs", default="rowscaled", choices=["rowscaled", "uniform"],
                    help="rowscaled: N(0,1) with log-uniform row scales; uniform: U[-1,1]")
    ap.add_argument("--p", type=int, default=64)
    ap.add_argument("--K", type=int, default=None, help="K of the schedule (2; 8 for nbody)")
    ap.add_argument("--form", default="split3_bf16")
    ap.add_argument("--compare", default="f32,split2_f16",
                    help="comma-separated forms timed beside the headline ('' to skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample (0 to skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for HBM counters)")
    ap.add_argument("--workload", default="step", choices=["step", "gemv", "complex", "nbody"],
                    help="step: the fwd+bwd product step (default); gemv: y = A.x alone "
                         "(A n x n FP32, HBM-bound; reports GB/s); complex: C = A.B on n x n "
                         "complex64 N(0,1) data (--form c32_split3_bf16, c32 or c32_split2_f16, compared with "
                         "the other two); "
                         "nbody: the all-pairs gravitational interaction of --bodies Plummer "
                         "bodies (FP32, ALU-bound; p = 64, K = 8 unless given)")
    ap.add_argument("--bodies", type=int, default=1 << 18, help="bodies of the nbody workload")
    ap.add_argument("--eps2", type=float, default=1e-4, help="softening of the nbody workload")
    a = ap.parse_args()
    if a.K is None:
        a.K = 8 if a.workload == "nbody" else 2
    if a.steps is None:
        a.steps = 200 if a.workload == "gemv" else 10
    return a


def step(hs, A, B, G, form, p, K):
    C = hs.hs_gemm(A, B, dtype=form, p=p, K=K)
    dA, dB = hs.hs_gemm_backward(A, B, G, dtype=form, p=p, K=K)
    return C, dA, dB


STORAGE = {"bf16": "bfloat16", "f16": "float16", "f64": "float64"}


def run_form(hs, torch, A, B, G, form, p, K, steps, warmup):
    """Times ``steps`` steps; returns (wall s, summed main-kernel ms,
    main-kernel launches, (C, dA, dB) of the last timed step)."""
    if form in STORAGE:   # the 16-bit and FP64 forms take inputs of their own type
        dt = getattr(torch, STORAGE[form])
        A, B, G = A.to(dt), B.to(dt), G.to(dt)
        torch.cuda.synchronize()
    for _ in range(warmup):
        step(hs, A, B, G, form, p, K)
    torch.cuda.synchronize()
    hs.hs_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        outs = step(hs, A, B, G, form, p, K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, launches = hs.hs_profile_end()
    return wall, kern_ms, launches, outs


def accuracy(outs, ref, n_elem=64):
    """err_row of the timed step's C, dA and dB on the rows the CPU baseline
    sampled, and err_elem (|dC| over the sum of absolute products) and
    err_term (|dC| over sqrt(k sum of squared products)) on the first
    ``n_elem`` of them."""
    import numpy as np
    import torch
    import oracle
    from oracle.metrics import err_elem, err_row, err_term
    rows_m, rows_k = ref["rows_m"], ref["rows_k"]
    A64, B64, G64 = ref["A"], ref["B"], ref["G"]
    e = rows_m[:n_elem], rows_k[:n_elem]
    # the operands of each output's sampled rows, as they multiply
    ops = {"C": lambda: (A64[e[0]], B64), "dA": lambda: (G64[e[0]], B64.T),
           "dB": lambda: (A64[:, e[1]].T, G64)}
    res = {}
    for name, out, rows in zip(("C", "dA", "dB"), outs, (rows_m, rows_m, rows_k)):
        got = out.index_select(0, torch.as_tensor(rows, device=out.device)).double().cpu().numpy()
        r = ref[name]
        X, Y = ops[name]()
        res[name] = {"err_row": err_row(got, r),
                     "err_elem": err_elem(got[:n_elem], r[:n_elem], oracle.absprod(X, Y)),
                     "err_term_u": err_term(got[:n_elem], r[:n_elem], oracle.sqprod(X, Y), X.shape[1]) / 2.0 ** -24}
    res["rows"] = ("%d sampled rows of each output (err_elem, err_term in units of 2^-24 on %d of them)"
                   % (len(rows_m), min(n_elem, len(rows_m))))
    return res


def cpu_baseline(A64, B64, G64, target_s):
    """The FP64 oracle on sampled rows of C, dA and dB (bounded sample).
    Returns (the baseline record, the oracle rows for the accuracy check)."""
    import oracle
    from paper_cs_9809105_amd import inputs
    m, k = A64.shape
    n = B64.shape[1]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate on one row per core of each product, then size the sample
    # (a multiple of the core count) to about target_s
    # one output row of C or dA costs 2 N Kd (resp. 2 N M) flops, of dB 2 M N
    cal = min(m, k, cores)
    rows_m = inputs.sample_rows(m, cal, seed=7)
    rows_k = inputs.sample_rows(k, cal, seed=7)
    t0 = time.perf_counter()
    oracle.gemm_rows(A64, B64, rows_m)
    oracle.grad_a_rows(G64, B64, rows_m)
    oracle.grad_b_rows(A64, G64, rows_k)
    t_cal = time.perf_counter() - t0
    nrows = int(cal * target_s / max(t_cal, 1e-6))
    nrows = max(cal, min(m, k, (nrows // cores) * cores))
    rows_m = inputs.sample_rows(m, nrows, seed=8)
    rows_k = inputs.sample_rows(k, nrows, seed=8)
    t0 = time.perf_counter()
    refC = oracle.gemm_rows(A64, B64, rows_m)
    refdA = oracle.grad_a_rows(G64, B64, rows_m)
    refdB = oracle.grad_b_rows(A64, G64, rows_k)
    dt = time.perf_counter() - t0
    flops = 2.0 * nrows * (n * k + n * k + m * n)
    # the same oracle on one thread, over a smaller sample (one row per core)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.gemm_rows(A64, B64, rows_m[:cal])
        oracle.grad_a_rows(G64, B64, rows_m[:cal])
        oracle.grad_b_rows(A64, G64, rows_k[:cal])
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    flops1 = 2.0 * cal * (n * k + n * k + m * n)
    rec = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
           "value_1thread": flops1 / dt1 / 1e12,
           "sample": "%d sampled rows of each of C, dA, dB (M=%d Kd=%d N=%d, FP64 triple loop, %.1f s); "
                     "1-thread figure on %d rows (%.1f s)" % (nrows, m, k, n, dt, cal, dt1)}
    ref = {"rows_m": rows_m, "rows_k": rows_k, "C": refC, "dA": refdA, "dB": refdB,
           "A": A64, "B": B64, "G": G64}
    return rec, ref


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "mm_kernel_split3_f32_n8192_traffic.json")


def kernel_source_sha256():
    """sha256 over the library's device and launch sources, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_cs_9809105_amd", "csrc")
    for name in ("hs_kernels.hip", "hs_internal.h", "hs_api.cpp"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(form, m, kd, n, p, K):
    """HBM bytes per main-kernel launch (FETCH_SIZE + WRITE_SIZE, calibrated
    against a plain device copy) from the committed rocprofv3 counter record,
    or None if there is no record for this workload or the kernels changed
    since it was taken."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_sha256():
        return None
    w = rec.get("workload", {})
    if (w.get("M"), w.get("Kd"), w.get("N"), w.get("p"), w.get("K")) != (m, kd, n, p, K):
        return None
    f = rec.get("forms", {}).get(form)
    return None if f is None else f["fetch_bytes"] + f["write_bytes"]


def gemv_main(args):
    """y = A . x, A n x n FP32 N(0, 1): one launch of the matrix-vector
    kernel per step, bounded by HBM (A is read once, 4 bytes per element).
    A 40 us kernel is shorter than one Python call into the library, so the
    timed steps are captured once into a HIP graph and replayed: the GPU
    then runs them back to back, and HIP events around the replay give the
    average launch time (kernel plus the graph's gap between launches)."""
    import torch
    import paper_cs_9809105_amd as hs
    from paper_cs_9809105_amd import inputs
    n, p, K = args.n, args.p, args.K
    A64 = inputs.normal((n, n), seed=inputs.BASE_SEED + 12)
    x64 = inputs.normal((n,), seed=inputs.BASE_SEED + 13)
    A = torch.from_numpy(A64).float().cuda()
    x = torch.from_numpy(x64).float().cuda()
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                   # eager warm-up before capture
        for _ in range(max(args.warmup, 1)):
            hs.hs_gemv(A, x, dtype="f32", p=p, K=K, out=y)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(args.steps):
            hs.hs_gemv(A, x, dtype="f32", p=p, K=K, out=y)
    graph.replay()                                  # warm replay
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    graph.replay()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, launches = ev0.elapsed_time(ev1), args.steps
    nbytes = 4.0 * (n * n + 2 * n)                  # A once, x and y
    avg = kern_ms / max(launches, 1)
    achieved = nbytes / (avg * 1e-3) / 1e9
    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        Ah = A.cpu().double().numpy()
        xh = x.cpu().double().numpy()
        reps, t_cpu = 0, 0.0
        t0 = time.perf_counter()
        while t_cpu < min(args.cpu_seconds, 5.0):
            yref = oracle.gemv(Ah, xh)
            reps += 1
            t_cpu = time.perf_counter() - t0
        cpu = {"value": nbytes * reps / t_cpu / 1e9, "unit": "GB/s", "kind": "oracle",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               "sample": "%d full %dx%d FP64 matrix-vector products (%.1f s)" % (reps, n, n, t_cpu)}
        from oracle.metrics import err_elem, err_row, err_term
        yg = y.double().cpu().numpy()[None, :]
        acc = {"f32": {"y": {"err_row": err_row(yg, yref[None, :]),
                             "err_elem": err_elem(yg, yref[None, :], oracle.gemv(abs(Ah), abs(xh))[None, :]),
                             "err_term_u": err_term(yg, yref[None, :], oracle.gemv(Ah * Ah, xh * xh)[None, :], n)
                             / 2.0 ** -24},
                       "rows": "all %d elements of the last timed y" % n}}
    else:
        acc = None
    print(json.dumps({
        "metric": "GB/s of y = A.x (A %dx%d FP32, read once)" % (n, n),
        "value": nbytes * args.steps / wall / 1e9, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "hyper-systolic matrix-vector product, A %dx%d N(0,1), x N(0,1)" % (n, n),
                   "M": n, "N": n, "p": p, "K": K, "form": "f32"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                     "frac": achieved / PEAK["hbm_gbs"], "traffic": None, "kernel": "gemv_kernel",
                     "avg_kernel_ms": avg, "launches": launches},
        "accuracy": acc,
        "cpu_baseline": cpu}))


def nbody_main(args):
    """The all-pairs gravitational interaction of n Plummer bodies (FP32):
    one hs_nbody call per step (interaction kernel and back-shift).  The
    interaction kernel is bound by the vector ALU: 20 flops per pair against
    the FP32 vector peak."""
    import torch
    import paper_cs_9809105_amd as hs
    from paper_cs_9809105_amd import inputs
    n, p, K, eps2 = args.bodies, args.p, args.K, args.eps2
    X64 = inputs.plummer(n, seed=inputs.BASE_SEED, unequal=False)
    X = torch.from_numpy(X64).float().cuda()
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        hs.hs_nbody(X, eps2, p=p, K=K, out=out)
    torch.cuda.synchronize()
    hs.hs_profile_begin()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        hs.hs_nbody(X, eps2, p=p, K=K, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, launches = hs.hs_profile_end()
    pairs = float(n) * (n - 1)
    avg = kern_ms / max(launches, 1)
    achieved = NBODY_FLOPS * pairs / (avg * 1e-3) / 1e12
    cpu = None
    if args.cpu_seconds > 0:
        import numpy as np
        import oracle
        Xh = X.cpu().double().numpy()
        e2 = float(np.float32(eps2))
        # calibrate on a small sample, then time one sample sized to last
        # about --cpu-seconds
        rows = 64
        t1 = time.perf_counter()
        oracle.nbody_rows(Xh, e2, inputs.sample_rows(n, rows, seed=9))
        t_cal = time.perf_counter() - t1
        rows = max(1, min(n, int(rows * args.cpu_seconds / max(t_cal, 1e-4))))
        idx = inputs.sample_rows(n, rows, seed=9)
        t1 = time.perf_counter()
        ref, scale = oracle.nbody_rows(Xh, e2, idx)
        t_cpu = time.perf_counter() - t1
        cpu = {"value": rows * (n - 1) / t_cpu / 1e9, "unit": "Ginteractions/s", "kind": "oracle",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               "value_tflops": NBODY_FLOPS * rows * (n - 1) / t_cpu / 1e12,
               "sample": "%d sampled bodies, each against all %d others (FP64 direct sum, %.1f s)"
                         % (rows, n - 1, t_cpu)}
        got = out.double().cpu().numpy()[idx]
        # acceleration error over the sum of the terms' lengths, potential
        # error relative to the potential (its terms have one sign)
        acc = {"f32": {"err_accel": float((np.abs(got[:, :3] - ref[:, :3]).max(axis=1) / scale).max()),
                       "err_phi": float((np.abs(got[:, 3] - ref[:, 3]) / np.abs(ref[:, 3])).max()),
                       "rows": "the %d sampled bodies of the last timed call" % rows}}
    else:
        acc = None
    print(json.dumps({
        "metric": "body-body interactions per second, all-pairs gravity of n=%d bodies (FP32)" % n,
        "value": pairs * args.steps / wall / 1e9, "unit": "Ginteractions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "two-array hyper-systolic all-pairs gravitational interaction, "
                               "n=%d Plummer-sphere bodies, equal masses, eps2=%g" % (n, eps2),
                   "n": n, "p": p, "K": K, "eps2": eps2, "form": "f32"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_F32_PEAK, "unit": "TFLOP/s",
                     "frac": achieved / VALU_F32_PEAK, "traffic": None, "kernel": "nbody_kernel",
                     "flops_per_interaction": NBODY_FLOPS, "avg_kernel_ms": avg, "launches": launches},
        "accuracy": acc,
        "cpu_baseline": cpu}))


def complex_main(args):
    """The fwd+bwd step on n x n complex64 data: C = A . B, dA = G . B^H,
    dB = A^H . G, each run as one real product of (complex as reals) and a
    2 x 2 block embedding; 8 n^3 useful real flops per product."""
    import numpy as np
    import torch
    import paper_cs_9809105_amd as hs
    from paper_cs_9809105_amd import inputs
    n, p, K = args.n, args.p, args.K
    form = args.form if args.form.startswith("c32") else "c32_split3_bf16"
    g = inputs.normal
    A64 = g((n, n), inputs.BASE_SEED + 20) + 1j * g((n, n), inputs.BASE_SEED + 21)
    B64 = g((n, n), inputs.BASE_SEED + 22) + 1j * g((n, n), inputs.BASE_SEED + 23)
    G64 = g((n, n), inputs.BASE_SEED + 24) + 1j * g((n, n), inputs.BASE_SEED + 25)
    A = torch.from_numpy(A64.astype(np.complex64)).cuda()
    B = torch.from_numpy(B64.astype(np.complex64)).cuda()
    G = torch.from_numpy(G64.astype(np.complex64)).cuda()

    def timed(fm, steps, warmup):
        for _ in range(warmup):
            step(hs, A, B, G, fm, p, K)
        torch.cuda.synchronize()
        hs.hs_profile_begin()
        t0 = time.perf_counter()
        for _ in range(steps):
            outs = step(hs, A, B, G, fm, p, K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms, launches = hs.hs_profile_end()
        return wall, ms / max(launches, 1), launches, outs[0]

    useful = 3 * 8.0 * n ** 3                      # per step
    base = {"c32": "f32", "c32_split3_bf16": "split3_bf16", "c32_split2_f16": "split2_f16"}

    def mfma_frac(fm, avg_ms):
        # one real product of 4 n^3 multiply-adds per complex product, times the form's MFMA products
        b = base[fm]
        return MFMA_PRODUCTS[b] * 8.0 * n ** 3 / (avg_ms * 1e-3) / 1e12 / PEAK[MFMA_PEAK_KEY[b]]

    wall, avg, launches_c, C_last = timed(form, args.steps, args.warmup)
    peak = PEAK[MFMA_PEAK_KEY[base[form]]]
    achieved = mfma_frac(form, avg) * peak
    comparison = None
    compares = [c for c in ("c32", "c32_split2_f16", "c32_split3_bf16") if c != form] if args.compare else []
    s2 = max(2, args.steps // 2)
    outs_cmp = {}
    for cf in compares:
        w2, a2, _, outs_cmp[cf] = timed(cf, s2, 1)
        comparison = comparison or {}
        comparison[cf] = {"value": useful * s2 / w2 / 1e12, "avg_main_kernel_ms": a2,
                          "mfma_frac": mfma_frac(cf, a2)}
    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        Ah = A.cpu().numpy().astype(np.complex128)
        Bh = B.cpu().numpy().astype(np.complex128)
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.complex_gemm_rows(Ah, Bh, inputs.sample_rows(n, cores, seed=7))
        t_cal = time.perf_counter() - t0
        nrows = max(cores, min(n, int(cores * args.cpu_seconds / max(t_cal, 1e-6)) // cores * cores))
        rows = inputs.sample_rows(n, nrows, seed=8)
        t0 = time.perf_counter()
        ref = oracle.complex_gemm_rows(Ah, Bh, rows)
        dt = time.perf_counter() - t0
        cpu = {"value": 8.0 * nrows * n * n / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
               "sample": "%d sampled rows of C (n=%d complex, FP64 parts, %.1f s)" % (nrows, n, dt)}
        from oracle.metrics import err_elem, err_row, err_term
        ne = min(16, nrows)
        absp = oracle.complex_absprod_rows(Ah, Bh, rows[:ne])
        sqp = oracle.complex_sqprod(Ah[rows[:ne]], Bh)
        acc = {}
        for fm, Cl in [(form, C_last)] + list(outs_cmp.items()):
            got = Cl.index_select(0, torch.as_tensor(rows, device=Cl.device)).cpu().numpy().astype(np.complex128)
            acc[fm] = {"C": {"err_row": err_row(got, ref), "err_elem": err_elem(got[:ne], ref[:ne], absp),
                             "err_term_u": err_term(got[:ne], ref[:ne], sqp, 2 * n) / 2.0 ** -24},
                       "rows": "%d sampled rows of the last timed C (err_elem on %d)" % (nrows, ne)}
    else:
        acc = None
    print(json.dumps({
        "metric": "TFLOP/s at n=%d complex64, fwd+bwd: %s" % (n, form),
        "value": useful * args.steps / wall / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": form,
        "data": "synthetic",
        "config": {"workload": "hyper-systolic complex C=A.B + dA=G.B^H + dB=A^H.G, square n=%d, "
                               "N(0,1) real and imaginary parts" % n,
                   "M": n, "Kd": n, "N": n, "p": p, "K": K, "form": form},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None, "kernel": "mm_kernel (main MFMA loop)",
                     "avg_kernel_ms": avg, "launches": launches_c},
        "comparison": comparison, "accuracy": acc, "cpu_baseline": cpu}))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the build runs on a single MI355X "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "gemv":
        return gemv_main(args)
    if args.workload == "complex":
        return complex_main(args)
    if args.workload == "nbody":
        return nbody_main(args)
    import numpy as np
    import torch
    import paper_cs_9809105_amd as hs
    from paper_cs_9809105_amd import inputs

    p, K = args.p, args.K
    if args.shape:
        m, kd, n = (int(x) for x in args.shape.split(","))
    else:
        m = kd = n = args.n
    gen = inputs.row_scaled if args.inputs == "rowscaled" else inputs.uniform
    A64 = gen((m, kd), seed=inputs.BASE_SEED + 2)
    B64 = gen((kd, n), seed=inputs.BASE_SEED + 3)
    G64 = inputs.normal((m, n), seed=inputs.BASE_SEED + 4)
    A = torch.from_numpy(A64).float().cuda()
    B = torch.from_numpy(B64).float().cuda()
    G = torch.from_numpy(G64).float().cuda()
    # the oracle sees exactly the stored fp32 values
    A64 = A.cpu().double().numpy()
    B64 = B.cpu().double().numpy()
    G64 = G.cpu().double().numpy()
    torch.cuda.synchronize()
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    useful = 3 * 2.0 * m * kd * n
    wall, kern_ms, launches, outs = run_form(hs, torch, A, B, G, args.form, p, K, args.steps, args.warmup)
    ms_step = wall * 1e3 / args.steps
    value = useful * args.steps / wall / 1e12
    avg_kernel_ms = kern_ms / max(launches, 1)
    # MFMA work of all timed main-kernel launches (three products per step,
    # each 2 m kd n times the form's MFMA products) over their summed time
    mfma_flops = MFMA_PRODUCTS[args.form] * 2.0 * m * kd * n * 3 * args.steps
    achieved = mfma_flops / (kern_ms * 1e-3) / 1e12
    peak = PEAK[MFMA_PEAK_KEY[args.form]]

    # the timed steps' outputs, kept on the GPU for the accuracy check
    outs_cmp = {}
    comparison = None
    for cf in [c for c in args.compare.split(",") if c]:
        s2 = max(2, args.steps // 2)
        w2, k2, l2, outs_cmp[cf] = run_form(hs, torch, A, B, G, cf, p, K, s2, 1)
        f2 = MFMA_PRODUCTS[cf] * 2.0 * m * kd * n * 3 * s2 / (k2 * 1e-3) / 1e12
        comparison = comparison or {}
        comparison[cf] = {"value": useful * s2 / w2 / 1e12, "ms_per_step": w2 * 1e3 / s2,
                          "avg_main_kernel_ms": k2 / max(l2, 1),
                          "mfma_frac": f2 / PEAK[MFMA_PEAK_KEY[cf]]}

    cpu = None
    acc = None
    if args.cpu_seconds > 0:
        cpu, ref = cpu_baseline(A64, B64, G64, args.cpu_seconds)
        acc = {args.form: accuracy(outs, ref)}
        for cf, o in outs_cmp.items():
            acc[cf] = accuracy(o, ref)

    square = m == kd == n
    shape_txt = "square n=%d" % n if square else "A %dx%d, B %dx%d" % (m, kd, kd, n)
    in_txt = ("row-scaled N(0,1) A and B" if args.inputs == "rowscaled" else "U[-1,1] A and B")
    out = {
        "metric": "TFLOP/s at n=8192: split-BF16 (FP32-accurate) vs plain FP32 GEMM; fwd+bwd",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.form, "data": "synthetic",
        "config": {"workload": "hyper-systolic C=A.B + dA=G.B^T + dB=A^T.G, %s, %s, N(0,1) G"
                               % (shape_txt, in_txt),
                   "M": m, "Kd": kd, "N": n, "p": p, "K": K, "form": args.form},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": recorded_traffic(args.form, m, kd, n, p, K),
                     "kernel": "mm_kernel (main MFMA loop)", "avg_kernel_ms": avg_kernel_ms,
                     "launches": launches},
        "comparison": comparison,
        "accuracy": acc,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
