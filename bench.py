"""Benchmark of the wall-corrected RPY blob-pair product and the GMRES solve on one GPU.

Headline (`value`): wall-RPY blob-pair interactions per second for one mobility
product u = M lambda over the 16,384-blob slab above a no-slip wall
(400a x 400a x [1.5a, 20a], minimum separation 2a, lambda ~ N(0,1)), FP32
pair sums with hi/lo positions and double accumulation across tiles.  One step
= one full product (all N^2 ordered pairs, self included) at a fixed
configuration, as in the solver: the positions are a context's state, set once
(the library prepares its own copy of them then), and every step multiplies
lambda; inputs resident on the GPU before timing.  The stateless entry point
(positions prepared inside every call) is reported beside it.

Also reported: the same product in FP64, the dominant kernel's roofline
(algorithmic flops / its HIP-event-timed duration), the CPU oracle on a bounded
sample, and the time per GMRES solve to 1e-6 on the 1,024-bacteria suspension
above a wall (FP32 pair sums, FP64 Krylov, block preconditioner).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve] [--pmc-copy]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic flops counted from the kernel expressions (FMA = 2, add/sub/mul = 1,
# reciprocal square root = 1; selects and compares 0; the Newton steps of the FP64
# reciprocal square root not counted; the overlap coefficients (r <= 2a), computed
# only when a wavefront holds an overlapping pair, not counted).  One-way: M_ij
# lambda_j for one ordered pair (target-parallel kernel, and the pairs inside the
# 256-blob diagonal blocks of the symmetric kernel).  Symmetric: one unordered pair
# applied both ways.
FLOPS_ONE_WAY = {("f32c", True): 104, ("f32c", False): 40, ("f64", True): 99,
                 ("f64", False): 34}
FLOPS_SYM = {("f32c", True): 132, ("f32c", False): 58, ("f64", True): 127,
             ("f64", False): 52}


# generalised RPY product of single-blob bodies (unbounded), same counting rules:
# (one ordered pair, one unordered pair applied both ways); FP32 adds the hi/lo
# displacement.  From 4,096 bodies on the library takes the symmetric form.
FLOPS_ROT = {"f64": (82, 145), "f32c": (88, 151)}


def rot_flops(M, prec, symmetric):
    one, both = FLOPS_ROT[prec]
    if not symmetric:
        return one * float(M) * M
    nb = [min(256, M - b) for b in range(0, M, 256)]
    p_diag = float(sum(n * n for n in nb))
    return both * (float(M) * M - p_diag) / 2.0 + one * p_diag


def algorithmic_flops(N, shape, prec="f32c", wall=True):
    """Flops of one product for the launch shape used (< 0: symmetric kernel)."""
    if shape > 0:
        return FLOPS_ONE_WAY[(prec, wall)] * float(N) * N
    nb = [min(256, N - b) for b in range(0, N, 256)]
    p_diag = float(sum(n * n for n in nb))
    p_off = (float(N) * N - p_diag) / 2.0
    return FLOPS_SYM[(prec, wall)] * p_off + FLOPS_ONE_WAY[(prec, wall)] * p_diag


def kernel_name(shape, prec="f32c"):
    if shape < 0:
        return f"pair_sym_{prec}_kernel<wall>"
    return f"pair_{prec}_kernel<wall>"


# MI355X published vector peaks: 256 CUs x 2.4 GHz x 256 FP32 (128 FP64) flop/clk/CU
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
HBM_TBS = 8.0
# HBM traffic of one pair product from the FETCH_SIZE / WRITE_SIZE runs recorded
# under profiles/ (KiB per dispatch, per launch shape the autotuner can pick),
# scaled by the counts of a 256 MiB copy; valid only for the kernel sources they
# were measured on (sha256 prefix of the listed files)
COPY_CAL = {"copy_fetch_kib": 131091.4, "copy_write_kib": 262144.0, "copy_kib": 262144.0}
TRAFFIC = {
    # target-parallel kernel: shape = source slices
    "target": {"src": ("pair.hip", "rpy_device.h"), "sha256_16": "022cc0a9700c3711",
               "by_shape": {16: (3858.0, 6144.0), 32: (3858.0, 12288.0),
                            64: (3858.0, 24576.0)}},
    # symmetric kernel: shape = -(source tiles per work item)
    "symmetric": {"src": ("pair_sym.hip", "rpy_device.h"), "sha256_16": "38aaae37f5705084",
                  "by_shape": {-1: (4415.2, 60864.0), -2: (4156.2, 36672.0),
                               -4: (4072.9, 24576.0), -8: (3917.4, 18624.0),
                               -16: (3967.9, 15648.0)}},
}


def measured_traffic(kind, shape):
    import hashlib

    t = TRAFFIC[kind]
    rec = t["by_shape"].get(shape)
    if rec is None or t["sha256_16"] is None:
        return None
    d = hashlib.sha256()
    for f in t["src"]:
        d.update(open(os.path.join(ROOT, "paper_2107_10800_amd", "csrc", f), "rb").read())
    if d.hexdigest()[:16] != t["sha256_16"]:
        return None
    fetch_kib, write_kib = rec
    c = COPY_CAL
    kib = (fetch_kib * c["copy_kib"] / c["copy_fetch_kib"]
           + write_kib * c["copy_kib"] / c["copy_write_kib"])
    return kib * 1024.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(sl, budget_s=20.0, u_gpu=None):
    """The oracle as it stands, timed on the host's cores: its compiled FP64 route
    (oracle/rpy_sum.c, plain loops, OpenMP over targets, every host thread) on
    the benchmark's product, target rows in blocks of 1,024 against all 16,384
    sources until the whole product is done or budget_s has passed (a bounded
    sample on small hosts).  With the GPU product u_gpu (N x 3) the sampled rows
    also give its relative error."""
    import numpy as np

    from oracle import rpy_c

    pos, lam = sl["pos"], sl["lam"]
    N = len(pos)
    rpy_c.load()
    done, elapsed, threads = 0, 0.0, 0
    rows = []
    block = 1024
    while done < N and elapsed < budget_s:
        tg = np.arange(done, min(N, done + block))
        t0 = time.perf_counter()
        u, threads = rpy_c.mobility_apply(pos, lam, 1.0, 1.0, True, targets=tg,
                                          return_threads=True)
        elapsed += time.perf_counter() - t0
        rows.append(u)
        done += len(tg)
    uo = np.vstack(rows)
    pairs = done * N
    what = "the whole product" if done == N else f"{done} target blobs x all {N} sources"
    res = {"value": pairs / elapsed, "unit": "pairs/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{what} of the 16,384-blob wall slab (float64, plain C loops over "
                     f"sources, OpenMP over targets, {threads} threads), {elapsed:.1f} s",
           "cpu_model": _cpu_model()}
    if u_gpu is not None:
        u = np.asarray(u_gpu).reshape(N, 3)[:done]
        res["gpu_rel_err_on_sample"] = float(np.linalg.norm(u - uo) / np.linalg.norm(uo))
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def matvec_bench_state(torch, arb, W, sl, precision, steps, warmup):
    """The product over a context's blobs at a fixed configuration (the solver's
    use: the positions are the state, set once; each step multiplies a new lambda):
    the headline."""
    N = len(sl["pos"])
    wl = W.loose_blobs(sl["pos"], sl["a"], sl["eta"], wall=True, name="wall slab")
    ctx = arb.context_for(wl, precision=precision)
    try:
        dev = torch.device("cuda")
        lam = torch.tensor(sl["lam"].ravel(), dtype=torch.float64, device=dev)
        u = torch.zeros_like(lam)
        stream = torch.cuda.Stream()
        sh = stream.cuda_stream
        torch.cuda.synchronize()
        for _ in range(max(warmup, 1)):          # includes the launch-shape autotune
            arb.arb_mobility_apply_dev(ctx, lam, u, stream=sh)
        torch.cuda.synchronize()
        arb.arb_profile_read(ctx)
        arb.arb_profile(ctx, True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        t0 = time.perf_counter()
        for _ in range(steps):
            arb.arb_mobility_apply_dev(ctx, lam, u, stream=sh)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1)
        kms, launches = arb.arb_profile_read(ctx)
        arb.arb_profile(ctx, False)
        slices = arb.arb_get_slices(ctx, N)
        out = u.cpu().numpy()
        return dict(ms_per_step=ms / steps, wall_s=wall, kernel_ms=kms / max(launches, 1),
                    launches=launches, slices=slices, u=out)
    finally:
        arb.arb_destroy(ctx)


def matvec_bench(torch, arb, sl, precision, steps, warmup):
    import numpy as np

    N = len(sl["pos"])
    ctx = arb.arb_create(precision=precision, wall=True)
    try:
        dev = torch.device("cuda")
        pos = torch.tensor(sl["pos"], dtype=torch.float64, device=dev)
        lam = torch.tensor(sl["lam"], dtype=torch.float64, device=dev)
        u = torch.zeros_like(lam)
        # an explicit stream: the library takes a null handle as "its own stream"
        stream = torch.cuda.Stream()
        sh = stream.cuda_stream
        torch.cuda.synchronize()
        for _ in range(max(warmup, 1)):          # includes the launch-shape autotune
            arb.arb_rpy_apply_dev(ctx, N, pos, lam, u, stream=sh)
        torch.cuda.synchronize()
        arb.arb_profile_read(ctx)
        arb.arb_profile(ctx, True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        t0 = time.perf_counter()
        for _ in range(steps):
            arb.arb_rpy_apply_dev(ctx, N, pos, lam, u, stream=sh)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1)
        kms, launches = arb.arb_profile_read(ctx)
        arb.arb_profile(ctx, False)
        slices = arb.arb_get_slices(ctx, N)
        out = u.cpu().numpy()
        return dict(ms_per_step=ms / steps, wall_s=wall, kernel_ms=kms / max(launches, 1),
                    launches=launches, slices=slices, u=out)
    finally:
        arb.arb_destroy(ctx)


def solve_roofline(wl, info, ms_measured):
    """Roofline time of one solve: the sum over its phases of algorithmic flops / peak or
    algorithmic bytes / HBM bandwidth, with the solver's own counts of products and
    preconditioner applications.  Products at the symmetric kernel's flops (each
    unordered pair once, the 256-blob diagonal blocks one way); preconditioner apply:
    M_pp^-1 (8 m^2 B) and Z_p (48 m B) per body read once; Krylov: CGS2 reads the basis
    twice per pass, 4 (j+1) n 8 B at Arnoldi step j, counted as one cycle; build:
    Cholesky, triangular inverse and product (m^3 / 3 flops each) per body at the FP64
    matrix-core peak.  Returns the phase times (ms) and roofline / measured."""
    import numpy as np

    N, n = wl.N, wl.n_unknowns
    m = 3 * np.diff(np.asarray(wl.blob_offset, np.int64)).astype(float)
    t32 = info["products_fp32"] * algorithmic_flops(N, -1, "f32c", wl.wall) / (PEAK_FP32_TFLOPS * 1e9)
    t64 = info["products_fp64"] * algorithmic_flops(N, -1, "f64", wl.wall) / (PEAK_FP64_TFLOPS * 1e9)
    pc_bytes = float(np.sum(8.0 * m * m + 48.0 * m))
    t_pc = info["precond_applies"] * pc_bytes / (HBM_TBS * 1e9)
    it = info["iterations"]
    t_kry = sum(4.0 * (j + 1) * n * 8.0 for j in range(it)) / (HBM_TBS * 1e9)
    t_build = float(np.sum(m ** 3)) / (PEAK_FP64_TFLOPS * 1e9)
    total = t32 + t64 + t_pc + t_kry + t_build
    return dict(products_fp32=info["products_fp32"], products_fp64=info["products_fp64"],
                precond_applies=info["precond_applies"],
                ms_pair_fp32=t32, ms_pair_fp64=t64, ms_precond_apply=t_pc, ms_krylov=t_kry,
                ms_build=t_build, ms_roofline=total, frac=total / ms_measured)


def solve_bench(torch, arb, wl, label, precision, tol=1e-6, reps=2):
    """Device solve of A y = b to tol (FP64 residual), preconditioner rebuilt each time."""
    ctx = arb.context_for(wl, precision=precision, tol=tol, restart=100, max_iter=1000)
    try:
        dev = torch.device("cuda")
        F = torch.tensor(wl.F.ravel(), dtype=torch.float64, device=dev)
        n = wl.n_unknowns
        y = torch.zeros(n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        sh = torch.cuda.Stream().cuda_stream
        rc, info = arb.arb_solve_dev(ctx, F, None, y, warm=False, stream=sh)   # warm-up
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, info = arb.arb_solve_dev(ctx, F, None, y, warm=False, stream=sh)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return dict(workload=f"{label}, N={wl.N}, M={wl.M}, Nc={wl.n_rows}, n={n}",
                    precision="f32c pair sums, f64 Krylov" if precision else "f64",
                    tol=tol, ms_per_solve=1e3 * min(times), iterations=info["iterations"],
                    rel_residual_fp64=info["rel_residual_fp64"],
                    precond_build_ms=info["t_build_ms"], status=rc,
                    pairs_per_matvec=int(wl.N) ** 2,
                    roofline=solve_roofline(wl, info, 1e3 * min(times)))
    finally:
        arb.arb_destroy(ctx)


def filament_bench(arb, W, reps=5):
    """Unbounded filament (20 rods x 4 blobs): FP64 solve to 1e-10, then one time step
    of 0.1 (solve, Euler update, reconstruction, correction run unconditionally),
    host-array entry points."""
    wl = W.filament()
    ctx = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-10)
    try:
        arb.arb_solve(ctx, wl.F)                                                 # warm-up
        ts, tt = [], []
        for _ in range(reps):
            arb.arb_set_state(ctx, wl.q, wl.theta)
            t0 = time.perf_counter()
            rc, U, phi, lam, info = arb.arb_solve(ctx, wl.F)
            t1 = time.perf_counter()
            arb.arb_set_state(ctx, wl.q, wl.theta)
            t2 = time.perf_counter()
            rs, q, th, U2, si = arb.arb_step_euler(ctx, wl.F, 0.1, delta=0.0, corr_tol=1e-10,
                                                   corr_max_iter=50, warm=False)
            t3 = time.perf_counter()
            ts.append(t1 - t0)
            tt.append(t3 - t2)
        return dict(workload=f"free filament, 20 rods x 4 blobs, unbounded, N={wl.N}, "
                             f"M={wl.M}, Nc={wl.n_rows}, n={wl.n_unknowns}",
                    precision="f64", tol=1e-10, ms_per_solve=1e3 * min(ts),
                    iterations=info["iterations"], rel_residual=info["rel_residual"], status=rc,
                    dt=0.1, ms_per_step=1e3 * min(tt), step_g_inf_rebuilt=si["g_inf_star"],
                    correction_iterations=si["corr_iterations"],
                    correction_residual=si["corr_residual"], step_g_inf=si["g_inf"])
    finally:
        arb.arb_destroy(ctx)


def timestep_bench(arb, W, n_bact=1024, dt=0.02, steps=3):
    """Explicit Euler steps of the bacteria suspension (Sec. 4.3): FP32 pair sums in
    GMRES to 1e-6 warm-started from the previous step, Euler update, reconstruction,
    check against delta = 1e-10 and correction to 1e-10; one cold step first; then
    one explicit midpoint step (App. C)."""
    import numpy as np

    wl = W.bacteria(n_bact=n_bact, seed=3)
    ctx = arb.context_for(wl, precision=arb.ARB_FP32C, tol=1e-6)
    try:
        rc, q, th, U, cold = arb.arb_step_euler(ctx, wl.F, dt, delta=1e-10, corr_tol=1e-10,
                                                warm=False)
        ts, infos = [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            rc, q, th, U, info = arb.arb_step_euler(ctx, wl.F, dt, delta=1e-10, corr_tol=1e-10,
                                                    warm=True)
            ts.append(time.perf_counter() - t0)
            infos.append(info)
        # one explicit midpoint step (App. C): two solves, the second warm-started
        t0 = time.perf_counter()
        rc_m, q, th, U, mid = arb.arb_step_midpoint(ctx, wl.F, dt, delta=1e-10, corr_tol=1e-10,
                                                    warm=True)
        t_mid = time.perf_counter() - t0
        # the rebuild alone (host entry point, synchronous)
        tr = []
        for _ in range(5):
            t0 = time.perf_counter()
            arb.arb_reconstruct(ctx)
            tr.append(time.perf_counter() - t0)
        return dict(workload=f"bacteria above a wall: {n_bact} x (42-blob head + 80-blob "
                             f"flagellum), N={wl.N}, M={wl.M}, Nc={wl.n_rows}, "
                             f"n={wl.n_unknowns}; dt={dt}",
                    precision="f32c pair sums, f64 Krylov", tol=1e-6,
                    ms_per_step=1e3 * float(np.mean(ts)), ms_per_step_min=1e3 * min(ts),
                    iterations_cold=cold["iterations"],
                    iterations_warm=[i["iterations"] for i in infos],
                    solve_ms_warm=[i["t_solve_ms"] for i in infos],
                    g_inf_rebuilt=[i["g_inf_star"] for i in infos],
                    corrected=[i["corrected"] for i in infos],
                    correction_iterations=[i["corr_iterations"] for i in infos],
                    g_inf_end=[i["g_inf"] for i in infos],
                    reconstruct_ms=1e3 * min(tr), status=rc,
                    midpoint_ms_per_step=1e3 * t_mid, midpoint_iterations=mid["iterations"],
                    midpoint_status=rc_m)
    finally:
        arb.arb_destroy(ctx)


def single_blob_bench(torch, arb, W, reps=5):
    """Single-blob bodies (Sec. 2.4, unbounded, FP64): the generalised RPY product on
    4,096 shells (172,032 bodies), and GMRES iterations to 1e-10 against the number of
    shells (Sec. 3.2.2; random forces and torques, and gravity) and of filaments
    (Sec. 3.2.1, 15 single blobs each, gravity, to 1e-8)."""
    out = {}
    wl = W.blob_shells(16)
    dev = torch.device("cuda")
    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    M = wl.M
    pairs = float(M) * M
    for prec, key in ((arb.ARB_FP64, "product"), (arb.ARB_FP32C, "product_fp32c")):
        ctx = arb.context_for(wl, precision=prec)
        try:
            F = torch.tensor(wl.F.ravel(), dtype=torch.float64, device=dev)
            UW = torch.zeros_like(F)
            arb.arb_body_mobility_apply_dev(ctx, F, UW, stream=sh)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for _ in range(reps):
                arb.arb_body_mobility_apply_dev(ctx, F, UW, stream=sh)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / reps
        finally:
            arb.arb_destroy(ctx)
        pname = "f64" if prec == arb.ARB_FP64 else "f32c"
        flops = rot_flops(M, pname, M >= 4096)
        tf = flops / (ms * 1e-3) / 1e12
        peak = PEAK_FP64_TFLOPS if prec == arb.ARB_FP64 else PEAK_FP32_TFLOPS
        out[key] = dict(workload=f"generalised RPY product, 4096 shells of 42 single blobs, "
                                 f"M={M}, unbounded", M=M, ms=ms,
                        pairs_per_s=pairs / (ms * 1e-3), flops_per_launch=flops,
                        flops_per_pair=FLOPS_ROT[pname], achieved_tflops=tf,
                        frac_of_peak=tf / peak, peak_tflops=peak,
                        kernel=f"rot_pair_sym_{pname}_kernel")
    out["product"]["frac_of_fp64_peak"] = out["product"]["frac_of_peak"]

    def solve(wl, tol, timed, prec=arb.ARB_FP64, pair_kernel=0):
        c = arb.context_for(wl, tol=tol, precision=prec, pair_kernel=pair_kernel)
        try:
            Fd = torch.tensor(wl.F.ravel(), dtype=torch.float64, device=dev)
            y = torch.zeros(wl.n_unknowns - 3 * wl.N, dtype=torch.float64, device=dev)
            if timed:
                arb.arb_solve_dev(c, Fd, None, y, warm=False, stream=sh)      # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, info = arb.arb_solve_dev(c, Fd, None, y, warm=False, stream=sh)
            torch.cuda.synchronize()
            return rc, info, 1e3 * (time.perf_counter() - t0)
        finally:
            arb.arb_destroy(c)

    scan = []
    for n_side in (1, 2, 4, 8, 16):
        for forcing in ("random", "gravity"):
            if n_side == 16 and forcing == "gravity":
                continue
            wl = W.blob_shells(n_side, forcing=forcing)
            rc, info, ms = solve(wl, 1e-10, n_side < 16)
            scan.append(dict(shells=n_side ** 3, forcing=forcing, M=wl.M, Nc=wl.n_rows,
                             n=6 * wl.M + wl.n_rows, iterations=info["iterations"],
                             rel_residual=info["rel_residual"], ms_per_solve=ms, status=rc))
            log(f"bench: {n_side ** 3} shells ({forcing}): {info['iterations']} iterations, "
                f"{ms:.1f} ms")
    out["shell_scan"] = scan
    # a practical tolerance (Sec. 3.2.1: 1e-3 - 1e-4) on 4,096 shells, FP64 against FP32
    # sums inside FP64 refinement
    prac = []
    wl = W.blob_shells(16)
    wlg = W.blob_shells(16, forcing="gravity")
    for w, prec, name in ((wl, arb.ARB_FP64, "f64"), (wl, arb.ARB_FP32C, "f32c"),
                          (wlg, arb.ARB_FP32C, "f32c gravity")):
        rc, info, ms = solve(w, 1e-4, False, prec)
        prac.append(dict(precision=name, tol=1e-4, iterations=info["iterations"],
                         rel_residual_fp64=info["rel_residual"], ms_per_solve=ms,
                         products_fp32=info["products_fp32"],
                         products_fp64=info["products_fp64"], status=rc))
        log(f"bench: 4096 shells to 1e-4, {name}: {info['iterations']} iterations, {ms:.1f} ms")
    out["shells4096_tol1e-4"] = prac
    fscan = []
    for k in (1, 2, 5, 10, 20):
        wl = W.blob_filaments(k, k)
        rc, info, ms = solve(wl, 1e-8, True)
        fscan.append(dict(filaments=k * k, M=wl.M, Nc=wl.n_rows, n=6 * wl.M + wl.n_rows,
                          iterations=info["iterations"], rel_residual=info["rel_residual"],
                          ms_per_solve=ms, status=rc))
    out["filament_scan"] = fscan
    # the fast product (ARB_PAIR_FMM, default order 6) on the 4,096 shells
    import numpy as np
    wl = W.blob_shells(16)
    F = torch.tensor(wl.F.ravel(), dtype=torch.float64, device=dev)
    ref = torch.zeros_like(F)
    c = arb.context_for(wl, precision=arb.ARB_FP64)
    try:
        arb.arb_body_mobility_apply_dev(c, F, ref, stream=sh)
        torch.cuda.synchronize()
    finally:
        arb.arb_destroy(c)
    ref_h = ref.cpu().numpy()
    fast = {}
    for prec, name, dense_ms in ((arb.ARB_FP32C, "float sums", out["product_fp32c"]["ms"]),
                                 (arb.ARB_FP64, "double sums", out["product"]["ms"])):
        c = arb.context_for(wl, precision=prec, pair_kernel=arb.ARB_PAIR_FMM)
        try:
            UW = torch.zeros_like(F)
            arb.arb_body_mobility_apply_dev(c, F, UW, stream=sh)
            st = arb.arb_fmm_get_stats(c)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                arb.arb_body_mobility_apply_dev(c, F, UW, stream=sh)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
        finally:
            arb.arb_destroy(c)
        err = float(np.abs(UW.cpu().numpy() - ref_h).max() / np.abs(ref_h).max())
        fast[name] = dict(ms=ms, dense_ms=dense_ms, speedup=dense_ms / ms,
                          max_rel_err_vs_dense_fp64=err, levels=st["levels"],
                          near_pairs=st["near_pairs"], m2l_pairs=st["m2l_pairs"])
        log(f"bench: 4096 shells, fast product ({name}) {ms:.2f} ms ({dense_ms / ms:.1f}x the "
            f"dense kernel), max error {err:.1e}")
    for tol, prec, name in ((1e-10, arb.ARB_FP64, "f64"), (1e-4, arb.ARB_FP32C, "f32c")):
        rc, info, ms = solve(wl, tol, True, prec, arb.ARB_PAIR_FMM)
        fast[f"solve_{name}_tol{tol:g}"] = dict(iterations=info["iterations"],
                                                rel_residual=info["rel_residual"],
                                                ms_per_solve=ms, status=rc)
        log(f"bench: 4096 shells to {tol:g} on the fast product ({name}): "
            f"{info['iterations']} iterations, {ms:.1f} ms")
    out["fast_product_4096_shells"] = fast
    return out


def fmm_bench(torch, arb, W, n_bact=8192, reps=10, log=log):
    """Fast wall mobility product (ARB_PAIR_FMM) on 8,192 bacteria above the wall
    (999,424 blobs): product time by Chebyshev order against the dense FP32 product,
    error against that product, tree statistics, and GMRES to 1e-6 on the fast
    operator (FP32 sums inside refinement by the double-sum variant)."""
    import numpy as np

    t0 = time.perf_counter()
    wl = W.bacteria(n_bact=n_bact, seed=3)
    t_gen = time.perf_counter() - t0
    dev = torch.device("cuda")
    lam = torch.tensor(np.random.default_rng(1).standard_normal(3 * wl.N), device=dev)
    u = torch.zeros(3 * wl.N, dtype=torch.float64, device=dev)
    ud = torch.zeros_like(u)
    # dense FP32 product (target-parallel kernel, one slice: no autotuning at this size)
    c = arb.context_for(wl, precision=arb.ARB_FP32C, pair_kernel=arb.ARB_PAIR_TARGET, slices=1)
    try:
        arb.arb_mobility_apply_dev(c, lam, ud)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        arb.arb_mobility_apply_dev(c, lam, ud)
        torch.cuda.synchronize()
        dense_ms = 1e3 * (time.perf_counter() - t0)
    finally:
        arb.arb_destroy(c)
    ref = ud.cpu().numpy()
    log(f"fmm bench: dense FP32 product {dense_ms:.0f} ms at N={wl.N}")
    rows = []
    for n in (4, 5, 6, 7):
        for prec, name in ((arb.ARB_FP32C, "float sums"), (arb.ARB_FP64, "double sums")):
            if n != 6 and prec == arb.ARB_FP64:
                continue
            c = arb.context_for(wl, precision=prec, pair_kernel=arb.ARB_PAIR_FMM, fmm_order=n)
            try:
                arb.arb_mobility_apply_dev(c, lam, u)
                st = arb.arb_fmm_get_stats(c)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    arb.arb_mobility_apply_dev(c, lam, u)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / reps
            finally:
                arb.arb_destroy(c)
            err = float(np.abs(u.cpu().numpy() - ref).max() / np.abs(ref).max())
            pairs = st["near_pairs"] + st["m2l_pairs"]
            tflops = pairs * FLOPS_ONE_WAY[("f32c", True)] / (ms * 1e-3) / 1e12
            rows.append(dict(order=n, sums=name, ms_per_product=ms, speedup_vs_dense=dense_ms / ms,
                             max_rel_err_vs_dense=err, levels=st["levels"], leaves=st["leaves"],
                             near_pairs=st["near_pairs"], m2l_pairs=st["m2l_pairs"],
                             tree_build_ms=st["build_ms"], pair_tflops=tflops,
                             frac_of_fp32_peak=tflops / PEAK_FP32_TFLOPS))
            log(f"fmm bench: n={n} {name}: {ms:.2f} ms ({dense_ms / ms:.0f}x dense), max error "
                f"{err:.1e}, L={st['levels']}, tree {st['build_ms']:.0f} ms, "
                f"{tflops:.1f} TFLOP/s of pair work")
    # GMRES on the fast operator
    c = arb.context_for(wl, precision=arb.ARB_FP32C, tol=1e-6, restart=100, max_iter=600,
                        pair_kernel=arb.ARB_PAIR_FMM)
    try:
        F = torch.tensor(wl.F.ravel(), dtype=torch.float64, device=dev)
        y = torch.zeros(wl.n_unknowns, dtype=torch.float64, device=dev)
        sh = torch.cuda.Stream().cuda_stream
        arb.arb_solve_dev(c, F, None, y, warm=False, stream=sh)      # builds tree and blocks
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = arb.arb_solve_dev(c, F, None, y, warm=False, stream=sh)
        torch.cuda.synchronize()
        solve_ms = 1e3 * (time.perf_counter() - t0)
    finally:
        arb.arb_destroy(c)
    log(f"fmm bench: solve {solve_ms:.0f} ms, {info['iterations']} iterations, residual "
        f"{info['rel_residual_fp64']:.1e}")
    # explicit Euler steps on the fast operator (Sec. 4.3): tree rebuilt per state,
    # GMRES warm-started from the previous step, reconstruction, check, correction
    c = arb.context_for(wl, precision=arb.ARB_FP32C, tol=1e-6, restart=100, max_iter=600,
                        pair_kernel=arb.ARB_PAIR_FMM)
    try:
        arb.arb_step_euler(c, wl.F, 0.02, delta=1e-10, corr_tol=1e-10, warm=False)
        steps = []
        for _ in range(2):
            t0 = time.perf_counter()
            rc_s, _, _, _, si = arb.arb_step_euler(c, wl.F, 0.02, delta=1e-10, corr_tol=1e-10,
                                                   warm=True)
            steps.append(dict(ms=1e3 * (time.perf_counter() - t0), iterations=si["iterations"],
                              rel_residual=si["rel_residual"], corrected=si["corrected"],
                              g_inf=si["g_inf"], tree_build_ms=arb.arb_fmm_get_stats(c)["build_ms"],
                              status=rc_s))
    finally:
        arb.arb_destroy(c)
    log(f"fmm bench: Euler steps {[round(x['ms']) for x in steps]} ms, iterations "
        f"{[x['iterations'] for x in steps]}")
    # unbounded: the diatom colonies on the fast operator (the dense solve is the
    # `diatoms` block)
    dw = W.diatoms()
    c = arb.context_for(dw, precision=arb.ARB_FP32C, tol=1e-6, restart=100, max_iter=1000,
                        pair_kernel=arb.ARB_PAIR_FMM)
    try:
        Fd = torch.tensor(dw.F.ravel(), dtype=torch.float64, device=dev)
        yd = torch.zeros(dw.n_unknowns, dtype=torch.float64, device=dev)
        arb.arb_solve_dev(c, Fd, None, yd, warm=False, stream=sh)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc_d, info_d = arb.arb_solve_dev(c, Fd, None, yd, warm=False, stream=sh)
        torch.cuda.synchronize()
        diatom_ms = 1e3 * (time.perf_counter() - t0)
        ud = torch.zeros(3 * dw.N, dtype=torch.float64, device=dev)
        lam_d = torch.tensor(np.random.default_rng(2).standard_normal(3 * dw.N), device=dev)
        arb.arb_mobility_apply_dev(c, lam_d, ud)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            arb.arb_mobility_apply_dev(c, lam_d, ud)
        torch.cuda.synchronize()
        diatom_prod_ms = 1e3 * (time.perf_counter() - t0) / reps
        dst = arb.arb_fmm_get_stats(c)
    finally:
        arb.arb_destroy(c)
    log(f"fmm bench: diatoms (unbounded, N={dw.N}) product {diatom_prod_ms:.2f} ms, solve "
        f"{diatom_ms:.0f} ms, {info_d['iterations']} iterations")
    return dict(workload=f"{n_bact} bacteria above a wall (42-blob head + 80-blob flagellum), "
                         f"N={wl.N} blobs, lambda ~ N(0,1)",
                seconds_generate=t_gen, dense_fp32_ms=dense_ms,
                dense_kernel="target-parallel FP32, one slice", products=rows,
                solve=dict(tol=1e-6, order=6, ms_per_solve=solve_ms,
                           iterations=info["iterations"],
                           rel_residual_fp64=info["rel_residual_fp64"],
                           products_fp64=info["products_fp64"],
                           products_fp32=info["products_fp32"],
                           precond_build_ms=info["t_build_ms"], status=rc),
                euler_steps=dict(dt=0.02, tol=1e-6, order=6, steps=steps),
                diatoms_unbounded=dict(N=dw.N, ms_per_product=diatom_prod_ms, levels=dst["levels"],
                                       ms_per_solve=diatom_ms, iterations=info_d["iterations"],
                                       rel_residual_fp64=info_d["rel_residual_fp64"],
                                       status=rc_d))


def learned_bench(torch, arb, W, n_bact=4096, n_train=100000, epochs=400, batch=1024, log=log):
    """Learned body-mobility preconditioner vs exact block and body-frame blocks."""
    import numpy as np

    from paper_2107_10800_amd import learned

    t0 = time.perf_counter()
    X, T = learned.make_dataset(n_train, seed=101)
    t_data = time.perf_counter() - t0
    sc = learned.scaling(X, T)
    ctx = arb.arb_create(precision=arb.ARB_FP64, wall=True)
    try:
        learned.load_model(ctx, W.mlp_init_weights(seed=6), sc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = learned.train(ctx, X, T, epochs=epochs, batch=batch, lr=2e-3, seed=7, log=log)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        params = arb.arb_mlp_get_params(ctx)
    finally:
        arb.arb_destroy(ctx)
    # held-out poses: the library's learned body mobilities (the blocks its learned
    # build uses) against its exact ones (the block build of Sec. 3.1)
    hold = W.bacterium_poses(1000, seed=202)
    c = arb.context_for(hold, precision=arb.ARB_FP64, precond=arb.ARB_PC_LEARNED)
    try:
        learned.load_model(c, params, sc)
        Ne = arb.arb_body_mobility(c)[0].reshape(-1, 6, 6)
        arb.arb_precond_build(c)
        Np = np.array([arb.arb_precond_block(c, p, 0)[1] for p in range(hold.M)])
    finally:
        arb.arb_destroy(c)
    err = np.linalg.norm(Np - Ne, axis=(1, 2)) / np.linalg.norm(Ne, axis=(1, 2))
    wl = W.bacteria(n_bact=n_bact, seed=5)
    dev = torch.device("cuda")
    F = torch.tensor(wl.F.ravel(), dtype=torch.float64, device=dev)
    y = torch.zeros(wl.n_unknowns, dtype=torch.float64, device=dev)
    out = {}
    cases = [("fp64_exact_block", arb.ARB_FP64, arb.ARB_PC_BLOCK),
             ("fp32c_exact_block", arb.ARB_FP32C, arb.ARB_PC_BLOCK),
             ("fp32c_learned", arb.ARB_FP32C, arb.ARB_PC_LEARNED),
             ("fp32c_body_frame", arb.ARB_FP32C, arb.ARB_PC_BODYFRAME)]
    for name, prec, pc in cases:
        c = arb.context_for(wl, precision=prec, tol=1e-6, restart=100, max_iter=600, precond=pc)
        try:
            learned.load_model(c, params, sc)
            torch.cuda.synchronize()
            sh = torch.cuda.Stream().cuda_stream
            arb.arb_solve_dev(c, F, None, y, warm=False, stream=sh)     # warm-up / autotune
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, info = arb.arb_solve_dev(c, F, None, y, warm=False, stream=sh)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            arb.arb_destroy(c)
        out[name] = dict(ms_per_solve=1e3 * dt, iterations=info["iterations"],
                         rel_residual_fp64=info["rel_residual_fp64"],
                         precond_build_ms=info["t_build_ms"], status=rc)
        log(f"learned bench {name}: {1e3 * dt:.0f} ms, {info['iterations']} iterations, "
            f"build {info['t_build_ms']:.1f} ms, residual {info['rel_residual_fp64']:.1e}")
    return dict(workload=f"{n_bact} bacteria above a wall, N={wl.N}, n={wl.n_unknowns}, "
                         f"GMRES to 1e-6 (FP64 residual)",
                training=dict(poses=int(len(X)), seconds_dataset=t_data, seconds_train=t_train,
                              epochs=epochs, batch=batch, final_batch_loss=hist[-1],
                              heldout_body_mobility_rel_err_median=float(np.median(err)),
                              heldout_body_mobility_rel_err_p95=float(np.percentile(err, 95))),
                solves=out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true",
                    help="skip comparing the timed product with the CPU baseline's oracle rows")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training the body-mobility network and the comparison of "
                         "preconditioners on 4,096 bacteria (about a minute)")
    ap.add_argument("--fmm-only", action="store_true",
                    help="run only the fast-product block (for profiling)")
    ap.add_argument("--no-fmm", action="store_true", help="skip the fast-product block")
    ap.add_argument("--single-blob-only", action="store_true",
                    help="run only the single-blob block (for profiling)")
    ap.add_argument("--pmc-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--matvec-only", action="store_true",
                    help="run only the headline FP32 product (autotune in the warm-up, then "
                         "--steps timed; for the counter runs) and print its timing")
    ap.add_argument("--solve-only", action="store_true",
                    help="run only the 1,024-bacteria FP32 solve (one warm-up, --steps timed; "
                         "for per-kernel profiles) and the filament solve")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2107_10800_amd import arb
    from paper_2107_10800_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    arb.load()
    if args.fmm_only:
        print(json.dumps({"fmm": fmm_bench(torch, arb, W, reps=args.steps)}), flush=True)
        return
    if args.single_blob_only:
        print(json.dumps({"single_blob": single_blob_bench(torch, arb, W)}), flush=True)
        return
    if args.solve_only:
        if args.pmc_copy:
            a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
            b = torch.empty_like(a)
            b.copy_(a)
            torch.cuda.synchronize()
            log("copy probe: 268435456 bytes read, 268435456 bytes written")
        out = {"gmres": solve_bench(torch, arb, W.bacteria(n_bact=1024, seed=3),
                                    "bacteria above a wall: 1024 x (42-blob head + 80-blob "
                                    "flagellum)", arb.ARB_FP32C, reps=max(1, min(args.steps, 3))),
               "filament": filament_bench(arb, W)}
        log(f"bench: solve {out['gmres']['ms_per_solve']:.1f} ms, "
            f"{out['gmres']['iterations']} iterations; filament "
            f"{out['filament']['ms_per_solve']:.2f} ms")
        print(json.dumps(out), flush=True)
        return
    sl = W.slab()
    N = len(sl["pos"])
    if args.pmc_copy:
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 268435456 bytes read, 268435456 bytes written")
    log(f"bench: wall slab N={N} f32c, {args.steps} steps")
    r32 = matvec_bench_state(torch, arb, W, sl, arb.ARB_FP32C, args.steps, args.warmup)
    log(f"bench: f32c {r32['ms_per_step']:.4f} ms/step, kernel {r32['kernel_ms']:.4f} ms, "
        f"slices {r32['slices']}")
    if args.matvec_only:
        print(json.dumps({k: v for k, v in r32.items() if k != "u"}), flush=True)
        return
    r64 = matvec_bench_state(torch, arb, W, sl, arb.ARB_FP64, max(args.steps // 4, 5), 2)
    log(f"bench: f64 {r64['ms_per_step']:.4f} ms/step")
    # the stateless entry point (positions prepared inside every call, blobs in the
    # order given, here the generator's random order)
    s32 = matvec_bench(torch, arb, sl, arb.ARB_FP32C, args.steps, args.warmup)
    log(f"bench: stateless f32c {s32['ms_per_step']:.4f} ms/step, kernel {s32['kernel_ms']:.4f} ms")
    pairs = float(N) * N
    value = pairs / (r32["ms_per_step"] * 1e-3)
    flops = algorithmic_flops(N, r32["slices"], "f32c")
    flops64 = algorithmic_flops(N, r64["slices"], "f64")
    achieved = flops / (r32["kernel_ms"] * 1e-3) / 1e12
    res = {
        "metric": "wall-RPY blob-pair interactions/s",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "wall-RPY mobility product, 16384 blobs in 400a x 400a x "
                               "[1.5a,20a] above a no-slip wall, min separation 2a, "
                               "lambda ~ N(0,1); one product per step at a fixed "
                               "configuration (positions set once as the context's state)",
                   "N": N, "pairs_per_step": int(pairs), "slices": r32["slices"],
                   "parity_rel_err_sampled": None},
        "roofline": {"bound": "alu",
                     "kernel": kernel_name(r32["slices"], "f32c"),
                     "flops_per_launch": flops,
                     "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "flops_per_pair": (FLOPS_SYM[("f32c", True)] if r32["slices"] < 0
                                        else FLOPS_ONE_WAY[("f32c", True)]),
                     "kernel_ms": r32["kernel_ms"],
                     "traffic": measured_traffic("symmetric" if r32["slices"] < 0 else "target",
                                                 r32["slices"]),
                     "traffic_unit": "bytes per launch (HBM, FETCH_SIZE + WRITE_SIZE of the "
                                     "launch shape timed, scaled by a 256 MiB copy)"},
        "stateless": {"value": pairs / (s32["ms_per_step"] * 1e-3), "unit": "pairs/s",
                      "ms_per_step": s32["ms_per_step"], "kernel_ms": s32["kernel_ms"],
                      "slices": s32["slices"],
                      "note": "arb_rpy_apply_dev: positions prepared inside every call, blobs "
                              "in the generator's random order"},
        "fp64": {"value": pairs / (r64["ms_per_step"] * 1e-3), "unit": "pairs/s",
                 "ms_per_step": r64["ms_per_step"], "kernel_ms": r64["kernel_ms"],
                 "kernel": kernel_name(r64["slices"], "f64"), "slices": r64["slices"],
                 "achieved_tflops": flops64 / (r64["kernel_ms"] * 1e-3) / 1e12,
                 "frac_of_fp64_peak": flops64 / (r64["kernel_ms"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS},
    }
    if not args.no_solve:
        log("bench: GMRES solve, bacteria 1024, f32c")
        res["gmres"] = solve_bench(torch, arb, W.bacteria(n_bact=1024, seed=3),
                                   "bacteria above a wall: 1024 x (42-blob head + 80-blob "
                                   "flagellum)", arb.ARB_FP32C)
        log(f"bench: solve {res['gmres']['ms_per_solve']:.1f} ms, "
            f"{res['gmres']['iterations']} iterations")
        log("bench: filament solve + correction, f64")
        res["filament"] = filament_bench(arb, W)
        log(f"bench: filament {res['filament']['ms_per_solve']:.2f} ms, "
            f"{res['filament']['iterations']} iterations, step {res['filament']['ms_per_step']:.2f} ms")
        log("bench: time steps, bacteria 1024, f32c")
        try:
            res["timestep"] = timestep_bench(arb, W)
            log(f"bench: time step {res['timestep']['ms_per_step']:.1f} ms, iterations "
                f"{res['timestep']['iterations_cold']} cold, "
                f"{res['timestep']['iterations_warm']} warm")
        except Exception as e:          # reported, not fatal to the headline line
            res["timestep"] = {"error": str(e)}
            log(f"bench: time steps failed: {e}")
        log("bench: single-blob bodies (generalised RPY), f64")
        try:
            res["single_blob"] = single_blob_bench(torch, arb, W)
            pr = res["single_blob"]["product"]
            p32 = res["single_blob"]["product_fp32c"]
            log(f"bench: generalised RPY product {pr['ms']:.1f} ms, {pr['pairs_per_s']:.3e} "
                f"pairs/s, {pr['frac_of_fp64_peak']:.3f} of FP64 peak; FP32 {p32['ms']:.1f} ms, "
                f"{p32['frac_of_peak']:.3f} of FP32 peak")
        except Exception as e:          # reported, not fatal to the headline line
            res["single_blob"] = {"error": str(e)}
            log(f"bench: single-blob bodies failed: {e}")
        log("bench: GMRES solve, diatom colonies, f32c")
        res["diatoms"] = solve_bench(torch, arb, W.diatoms(),
                                     "256 unbounded diatom colonies of 5-40 plates (15 x 3 blobs) "
                                     "with sliding links", arb.ARB_FP32C, reps=1)
        log(f"bench: diatoms {res['diatoms']['ms_per_solve']:.1f} ms, "
            f"{res['diatoms']['iterations']} iterations")
    if not args.no_solve and not args.no_fmm:
        log("bench: fast product, 8192 bacteria")
        try:
            res["fmm"] = fmm_bench(torch, arb, W)
        except Exception as e:          # reported, not fatal to the headline line
            res["fmm"] = {"error": str(e)}
            log(f"bench: fast product failed: {e}")
    if not args.no_solve and not args.no_learned:
        log("bench: learned preconditioner, 4096 bacteria")
        try:
            res["learned"] = learned_bench(torch, arb, W)
        except Exception as e:          # reported, not fatal to the headline line
            res["learned"] = {"error": str(e)}
            log(f"bench: learned preconditioner failed: {e}")
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(sl, u_gpu=None if args.no_check else r32["u"])
        # the oracle's sampled rows against the timed FP32 product
        res["config"]["parity_rel_err_sampled"] = res["cpu_baseline"].pop("gpu_rel_err_on_sample",
                                                                          None)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
