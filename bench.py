"""Benchmark of the matrix-free SIMP hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one outer iteration of the first-order bilevel method on the
128x64x64 hex8 cantilever (524,288 elements, 1,635,075 DOFs): density
filter, SIMP scaling and Jacobi diagonal, 8 warm-started Jacobi-PCG steps
(each one K(rho) p product), sensitivity u_e^T KE u_e, filter transpose,
mean-projected gradient step and FP64 projection onto the volume box.
Inputs are seeded synthetic data resident in HBM before timing starts.
Prints ONE JSON line (rank 0).  The value is outer iterations per second
of the FP32 path (FP32 storage and arithmetic, FP64 reductions), the K
timed iterations run in one fbto_outer_steps call (`one_call_per_iteration`
times them one fbto_outer_step call each); the same
line carries the FP64 path, the K(rho)u rate in GDOF/s with its roofline
fraction, the time to a fixed residual (FP32 + FP64 refinement vs FP64),
and the CPU oracle timed on the host cores.  `roofline` is that of the
kernel that dominates the step, the fused Jacobi-PCG step
(`fused_step_sizes` gives the same kernel on the 256x128x128 and
384x192x192 grids); `outer_roofline` sets the whole iteration against its
algorithmic bytes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "K(ρ)u GDOF/s + TO outer iters/s, 128x64x64 hex, mixed vs FP64 at fixed err"
HBM_PEAK_GBS = 8000.0
ALPHA0_CFG3 = 0.0016591384929631413      # tests/golden/alpha0.json (oracle-generated)
KERNEL_SOURCES = ("paper_2204_06204_amd/csrc/kernels.hip", "paper_2204_06204_amd/csrc/device.h")
COPY_BYTES = 256 << 20                   # calibration copy of the HBM counters
KRYLOV_DEGREE = 20                       # D of Alg. 3's Krylov preconditioner (the paper's choice)
PGD_RTOL = 1e-5                          # low-level tolerance of the exact-solve baseline (FP32 solves)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key: str, summary: str = "apply_K_pmc.json"):
    """HBM bytes (fetch + write) per launch of the named kernel from the
    committed rocprofv3 PMC summary, scaled by the calibration copy, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    for name, v in d.get("kernels", {}).items():
        if kernel_key in name and v.get("fetch_bytes") is not None and v.get("write_bytes") is not None:
            return v["fetch_bytes"] + v["write_bytes"]
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--apply-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fixed-err", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-sizes", action="store_true",
                    help="skip the K(rho)u timings at 256x128x128 and 384x192x192")
    ap.add_argument("--profile-only", choices=["apply", "outer", "cpfbto", "project", "fused_large", "plane"],
                    default=None,
                    help="run only a short loop of one kind (for rocprofv3)")
    return ap.parse_args()


def outer_loop(g, p, dtype, steps, warmup, torch, krylov=None, exact_rtol=None, alpha0=None, true_obj=True,
               multi=False):
    """Times `steps` outer iterations after `warmup` untimed ones (Alg. 1
    with Jacobi-PCG, or with krylov=D Alg. 3 with the Krylov preconditioner
    of degree D, beta = 1, or with exact_rtol projected gradient descent
    with the low-level problem solved to that relative residual).  multi
    (Alg. 1): the warm-up iterations in one fbto_outer_steps call, the timed
    ones in another; else one fbto_outer_step call per iteration."""
    dev = torch.device("cuda:0")
    x = g.project_volume(torch.tensor(p.x0, dtype=dtype, device=dev), lo=0.0, hi=1.0, vmax=p.vmax)
    u = torch.zeros(p.ndof, dtype=dtype, device=dev)
    f = torch.tensor(p.loads[0], dtype=dtype, device=dev)
    info = torch.zeros(8, dtype=torch.float64, device=dev)
    k = 1
    a0 = ALPHA0_CFG3 if alpha0 is None else alpha0
    if multi:
        assert krylov is None and exact_rtol is None
        infos = torch.zeros(8 * max(steps, warmup, 1), dtype=torch.float64, device=dev)
        if warmup:
            g.outer_steps(x, u, f, k, warmup, a0, p.inner_steps, 0.0, p.vmax, info=infos)
            k += warmup
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.outer_steps(x, u, f, k, steps, a0, p.inner_steps, 0.0, p.vmax, info=infos)
        k += steps
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        inf = infos[8 * (steps - 1):8 * steps].cpu().tolist()
        return dt, {"compliance": inf[0], "dx_inf": inf[1], "r_inf": inf[2], "lambda": inf[3],
                    "volume": inf[4], "status": inf[6], "k_last": k - 1,
                    "true_compliance": true_compliance(g, p, x, torch) if true_obj else None}
    def step(k):
        if exact_rtol is not None:
            g.outer_step(x, u, f, k, a0, 100000, 0.0, p.vmax, info=info, method="exact", rtol=exact_rtol)
        elif krylov is None:
            g.outer_step(x, u, f, k, a0, p.inner_steps, 0.0, p.vmax, info=info)
        else:
            g.outer_step(x, u, f, k, a0, krylov, 0.0, p.vmax, info=info, method="krylov", beta=1.0)
    for _ in range(warmup):
        step(k)
        k += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(k)
        k += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    inf = info.cpu().tolist()
    return dt, {"compliance": inf[0], "dx_inf": inf[1], "r_inf": inf[2], "lambda": inf[3],
                "volume": inf[4], "status": inf[6], "k_last": k - 1,
                "true_compliance": true_compliance(g, p, x, torch) if true_obj else None}


def true_compliance(g, p, x, torch):
    """f^T K(C(x))^-1 f at design x, solved in FP64 with FP32 inner solves and
    FP64 refinement to a relative residual of 1e-9 (the objective the inexact
    low-level solves track)."""
    rho = g.filter(x.double().contiguous())
    f = torch.tensor(p.loads[0], dtype=torch.float64, device=x.device)
    u = torch.zeros_like(f)
    g.solve_refined(rho, f, u, 1e-9, 100, 20000, inner_dtype=torch.float32, inner_rtol=1e-3)
    return float(torch.dot(f, u))


def apply_timing(g, p, dtype, reps, torch, cold=False, binary=False):
    """Average duration of one fbto_apply_K launch, from HIP events recorded
    on the stream the kernel runs on (the current torch stream).  `binary`:
    a near-binary density (rho_min or 1, 30% solid) instead of the seeded
    U[0.2, 0.4] field, to show the time does not depend on the data."""
    dev = torch.device("cuda:0")
    rho = torch.tensor(p.x0, dtype=dtype, device=dev)
    if binary:
        sel = torch.rand(rho.shape, generator=torch.Generator(device=dev).manual_seed(3), device=dev) < 0.3
        rho = torch.where(sel, torch.ones_like(rho), torch.full_like(rho, 1e-3))
    u = torch.randn(p.ndof, dtype=dtype, device=dev, generator=torch.Generator(device=dev).manual_seed(1))
    y = torch.empty_like(u)
    st = torch.cuda.current_stream()
    for _ in range(10):
        g.apply_K(rho, u, y)
    if not cold:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            g.apply_K(rho, u, y)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps
    # cold: overwrite a 1 GiB buffer (4x the 256 MB Infinity Cache) between launches
    scratch = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    tot = 0.0
    n = max(10, reps // 10)
    for _ in range(n):
        scratch.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        g.apply_K(rho, u, y)
        e1.record(st)
        torch.cuda.synchronize()
        tot += e0.elapsed_time(e1) * 1e-3
    return tot / n


def fused_step_timing(g, p, torch, reps=20, n1=9, n2=41):
    """Average duration of one fused CG step launch (FP32), the kernel that
    dominates the outer iteration.  A solve of n steps runs n - 1 fused
    launches beside a fixed set of other kernels, so the difference of the
    times of n2- and n1-step solves (HIP events on the launch stream) over
    n2 - n1 is one fused launch.  The two solves alternate and the medians
    of their times are taken, so that clock drift cancels."""
    import statistics
    dev = torch.device("cuda:0")
    rho = torch.tensor(p.x0, dtype=torch.float32, device=dev)
    f = torch.tensor(p.loads[0], dtype=torch.float32, device=dev)
    u = torch.zeros_like(f)
    st = torch.cuda.current_stream()
    times = {n1: [], n2: []}
    for i in range(reps + 2):
        for n in (n2, n1):
            u.zero_()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            g.inner_solve(rho, f, u, n, rtol=0.0)
            e1.record(st)
            torch.cuda.synchronize()
            if i >= 2:
                times[n].append(e0.elapsed_time(e1) * 1e-3)
    return (statistics.median(times[n2]) - statistics.median(times[n1])) / (n2 - n1)


def fixed_error(g, p, torch, rtol=1e-8):
    """Time to ||f - K u|| <= rtol ||f|| from u = 0 at the seeded density:
    FP64 Jacobi-PCG vs FP32 Jacobi-PCG with FP64 iterative refinement."""
    dev = torch.device("cuda:0")
    rho = torch.tensor(p.x0, dtype=torch.float64, device=dev)
    f = torch.tensor(p.loads[0], dtype=torch.float64, device=dev)
    out = {}
    info = torch.zeros(8, dtype=torch.float64, device=dev)
    u = torch.zeros_like(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.inner_solve(rho, f, u, 200000, rtol=rtol, info=info)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    i64 = info.cpu().tolist()
    c64 = float(torch.dot(f, u))
    u2 = torch.zeros_like(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nref = g.solve_refined(rho, f, u2, rtol, 100, 20000, inner_dtype=torch.float32, inner_rtol=1e-3,
                           info=info)
    torch.cuda.synchronize()
    tmix = time.perf_counter() - t0
    imix = info.cpu().tolist()
    cmix = float(torch.dot(f, u2))
    out["rtol"] = rtol
    out["fp64_pcg"] = {"seconds": t64, "pcg_steps": i64[3], "rel_residual": i64[0] / i64[2]}
    out["fp32_pcg_fp64_refine"] = {"seconds": tmix, "inner_steps_taken": imix[3], "refinements": nref,
                                   "inner_rtol": 1e-3,
                                   "rel_residual": imix[0] / imix[2],
                                   "compliance_rel_diff_vs_fp64": abs(cmix - c64) / abs(c64)}
    out["speedup_mixed_vs_fp64"] = t64 / tmix if tmix > 0 else None
    return out


def outer_sizes(torch):
    """Outer iterations/s of the two smaller workloads as configured (16x8x8
    with 5 PCG steps, 64x32x32 with 8), FP32 and FP64, step sizes from
    tests/golden/alpha0.json."""
    import synth
    from paper_2204_06204_amd.grid import Grid
    a0 = json.load(open(os.path.join(ROOT, "tests", "golden", "alpha0.json")))
    out = {}
    for name in ("cfg1", "cfg2"):
        p = synth.config(name)
        g = Grid.from_problem(p)
        for dtype, tag in ((torch.float32, "fp32"), (torch.float64, "fp64")):
            dt, st = outer_loop(g, p, dtype, 100, 10, torch, alpha0=a0[name], true_obj=False)
            out[f"{name}_{tag}"] = {"outer_iter_s": 100 / dt, "grid": [p.nx, p.ny, p.nz],
                                    "inner_steps": p.inner_steps, "compliance": st["compliance"]}
        g.close()
    return out


def fixed_error_cfg4(torch):
    """The fixed-error comparison on the 256x128x128 bridge (supports at the
    two bottom edges, uniform traction on the top face), seeded density."""
    import synth
    from paper_2204_06204_amd.grid import Grid
    p = synth.config("cfg4")
    g = Grid.from_problem(p)
    out = fixed_error(g, p, torch)
    g.close()
    torch.cuda.empty_cache()
    return out


def apply_sizes(torch):
    """K(rho)u at the two larger workloads (bridge 256x128x128, cantilever
    384x192x192 with 1 and 4 load cases): GDOF/s and HBM fraction of the
    algorithmic bytes, warm, from HIP events on the launch stream."""
    import synth
    from paper_2204_06204_amd.grid import Grid
    out = {}
    dev = torch.device("cuda:0")
    for name, nrhs_list in (("cfg4", (1,)), ("cfg5", (1, 4))):
        p = synth.config(name)
        g = Grid.from_problem(p, max_rhs=max(nrhs_list))
        st = torch.cuda.current_stream()
        for dtype, b in ((torch.float32, 4), (torch.float64, 8)):
            for nr in nrhs_list:
                if nr > 1 and dtype == torch.float64:
                    continue
                rho = torch.tensor(p.x0, dtype=dtype, device=dev)
                u = torch.randn(nr * p.ndof, dtype=dtype, device=dev,
                                generator=torch.Generator(device=dev).manual_seed(1))
                y = torch.empty_like(u)
                for _ in range(3):
                    g.apply_K(rho, u, y)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                for _ in range(20):
                    g.apply_K(rho, u, y)
                e1.record(st)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) * 1e-3 / 20
                nbytes = 2 * nr * p.ndof * b + p.E * b
                out[f"{name}_{'fp32' if b == 4 else 'fp64'}_rhs{nr}"] = {
                    "us": t * 1e6, "gdof_s": nr * p.ndof / t / 1e9, "hbm_frac": nbytes / t / 1e9 / HBM_PEAK_GBS,
                    "grid": [p.nx, p.ny, p.nz]}
                del rho, u, y
        g.close()
        torch.cuda.empty_cache()
    return out


def fused_sizes(torch):
    """The fused CG step (FP32, one load case) on the two larger grids,
    timed as in the headline roofline: HIP events around solves of 41 and 9
    steps; HBM fraction of the same algorithmic bytes (11*3N*4 + N + 4E)."""
    import synth
    from paper_2204_06204_amd.grid import Grid
    out = {}
    for name in ("cfg4", "cfg5"):
        p = synth.config(name)
        g = Grid.from_problem(p, max_rhs=1)
        t = fused_step_timing(g, p, torch, reps=5)
        nbytes = 11 * p.ndof * 4 + p.N + 4 * p.E
        out[name] = {"us": t * 1e6, "hbm_frac": nbytes / t / 1e9 / HBM_PEAK_GBS, "bytes": nbytes,
                     "grid": [p.nx, p.ny, p.nz]}
        g.close()
        torch.cuda.empty_cache()
    return out


def projection_timing(torch, reps=20):
    """The two device projections onto {0 <= x <= 1, sum x <= vmax}
    (fbto_project_volume: safeguarded Newton; fbto_project_volume_sorted:
    Alg. 4 as a radix sort and scans) at 128x64x64 and 384x192x192, FP32
    and FP64, from HIP events on the launch stream.  The input is a
    gradient step from a U[0.2, 0.4] density (the multiplier is positive).
    Streaming bytes of the sorted path per element, with b bytes per value:
    per 8-bit pass histogram b + scatter 2b (the first pass reads y itself);
    prefix sums b + b + 8; bracket b (its searches hit cache); clamp 2b."""
    import numpy as np
    import synth
    from paper_2204_06204_amd.grid import Grid
    out = {}
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    for name, shape, vf in (("128x64x64", (128, 64, 64), 0.25), ("384x192x192", (384, 192, 192), 0.1)):
        p = synth.cantilever(*shape, volfrac=vf, filter_radius=1.0, outer_iters=1, inner_steps=1)
        g = Grid.from_problem(p)
        rng = np.random.default_rng(5)
        y64 = rng.uniform(0.2, 0.4, p.E) - 0.05 * rng.normal(0.0, 1.0, p.E)
        for dtype, b in ((torch.float32, 4), (torch.float64, 8)):
            y = torch.tensor(y64, dtype=dtype, device=dev)
            x = torch.empty_like(y)
            lam = torch.zeros(2, dtype=torch.float64, device=dev)
            rec = {}
            for i, method in enumerate(("newton", "sort")):
                for _ in range(3):
                    g.project_volume(y, x, 0.0, 1.0, p.vmax, lam=lam[i:i + 1], method=method)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                for _ in range(reps):
                    g.project_volume(y, x, 0.0, 1.0, p.vmax, lam=lam[i:i + 1], method=method)
                e1.record(st)
                torch.cuda.synchronize()
                rec[f"{method}_us"] = e0.elapsed_time(e1) * 1e3 / reps
            passes = 8 * b // 8
            nbytes = p.E * (passes * 3 * b + 2 * b + 8 + b + 2 * b)
            rec["sort_bytes"] = nbytes
            rec["sort_hbm_frac"] = nbytes / (rec["sort_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
            lv = lam.cpu().tolist()
            rec["lambda_newton"], rec["lambda_sort"] = lv[0], lv[1]
            out[f"{name}_{'fp32' if b == 4 else 'fp64'}"] = rec
            del y, x
        g.close()
        torch.cuda.empty_cache()
    return out


def optimality_history(g, p, torch):
    """The true objective l(v_k) and the high-level error Delta^v_k of Thm. 1
    (fbto_optimality, FP64 solve to a relative residual of 1e-8) along runs
    of the three methods on the 128x64x64 workload: FBTO (Alg. 1, 8 PCG
    steps), CPFBTO (Alg. 3, D = 20) and PGD with exact low-level solves,
    every few iterations; alpha_k = alpha0 k^(-3/4)."""
    dev = torch.device("cuda:0")
    f64 = torch.tensor(p.loads[0], dtype=torch.float64, device=dev)
    out = {}
    for name, iters, every in (("fbto", 60, 10), ("cpfbto", 30, 5), ("pgd", 10, 2)):
        x = g.project_volume(torch.tensor(p.x0, dtype=torch.float32, device=dev), lo=0.0, hi=1.0, vmax=p.vmax)
        u = torch.zeros(p.ndof, dtype=torch.float32, device=dev)
        f = f64.float()
        info = torch.zeros(8, dtype=torch.float64, device=dev)
        rows = []
        t_run = 0.0
        for k in range(1, iters + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "fbto":
                g.outer_step(x, u, f, k, ALPHA0_CFG3, p.inner_steps, 0.0, p.vmax, info=info)
            elif name == "cpfbto":
                g.outer_step(x, u, f, k, ALPHA0_CFG3, KRYLOV_DEGREE, 0.0, p.vmax, info=info, method="krylov")
            else:
                g.outer_step(x, u, f, k, ALPHA0_CFG3, 100000, 0.0, p.vmax, info=info, method="exact", rtol=PGD_RTOL)
            torch.cuda.synchronize()
            t_run += time.perf_counter() - t0
            if k % every == 0 or k == 1:
                alpha_k = ALPHA0_CFG3 * (k + 1) ** -0.75
                m = g.optimality(x.double(), u.double(), f64, alpha_k, 0.0, p.vmax, rtol=1e-8).cpu().tolist()
                rows.append({"k": k, "seconds": t_run, "l": m[0], "delta_v": m[1], "delta_u": m[2],
                             "rel_residual": m[3], "status": m[4], "compliance_inexact": float(info[0])})
        out[name] = rows
    return out


def plane_path(torch):
    """Alg. 3 (D = 20, beta = 1, box [0.1, 1], eta = 3, 7x7 Gaussian filter) on
    plane cantilevers at two of the paper's table shapes, FP32 and FP64,
    seconds per outer iteration beside the paper's figure for the shape
    (its hardware: a GTX 1060 mobile GPU)."""
    import synth
    from paper_2204_06204_amd.grid import PlaneGrid
    a0 = json.load(open(os.path.join(ROOT, "tests", "golden", "alpha0.json")))
    paper = {"plane_a": 0.040, "plane_e": 0.011}
    out = {}
    dev = torch.device("cuda:0")
    for name in ("plane_a", "plane_e"):
        p = synth.plane_config(name)
        g = PlaneGrid.from_problem(p)
        rec = {"grid": [p.ny, p.nx], "volfrac": p.volfrac, "elements": p.E, "dofs": p.ndof,
               "paper_s_per_iter": paper[name], "paper_hardware": "GTX 1060 mobile (1280 cores), 2D regular grid"}
        alpha0 = a0.get(name, a0["plane_a"])
        for dtype, tag in ((torch.float32, "fp32"), (torch.float64, "fp64")):
            x = torch.full((p.E,), p.volfrac, dtype=dtype, device=dev)
            u = torch.zeros(p.ndof, dtype=dtype, device=dev)
            f = torch.tensor(p.loads[0], dtype=dtype, device=dev)
            info = torch.zeros(8, dtype=torch.float64, device=dev)
            n = 50
            for k in range(1, 6):
                g.outer_step(x, u, f, k, alpha0, p.degree, p.lo, p.vmax, info=info, method="krylov", beta=p.beta)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(6, 6 + n):
                g.outer_step(x, u, f, k, alpha0, p.degree, p.lo, p.vmax, info=info, method="krylov", beta=p.beta)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / n
            rec[f"{tag}_s_per_iter"] = dt
            rec[f"{tag}_speedup_vs_paper"] = paper[name] / dt
            rec[f"{tag}_status"] = float(info[6])
        out[name] = rec
        g.close()
    return out


def cpu_baseline(p, seconds):
    """The CPU FP64 oracle (as it stands) running outer iterations of the same
    workload on the host cores for about `seconds`."""
    import numpy as np
    import threadpoolctl
    import oracle
    from oracle.outer import OuterContext, outer_step_ref
    ctx = OuterContext(p.nx, p.ny, p.nz, p.filter_radius, p.fixed_mask, p.springs, use_csr=False)
    x = oracle.project_volume_ref(p.x0, 0.0, 1.0, p.vmax)
    u = np.zeros_like(p.loads)
    n, k = 0, 1
    t0 = time.perf_counter()
    while True:
        x, u, rec, _ = outer_step_ref(ctx, x, u, p.loads, k, ALPHA0_CFG3, p.inner_steps, 0.0, 1.0, p.vmax)
        n += 1
        k += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    blas = max((d.get("num_threads", 1) for d in threadpoolctl.threadpool_info()), default=1)
    return {"value": n / dt, "unit": "outer_iter/s", "cores": int(blas), "kind": "oracle",
            "sample": f"{n} outer iteration(s) of the 128x64x64 workload from the projected seeded "
                      f"density (NumPy/SciPy FP64 element-loop K u, 8 PCG steps each), {dt:.1f} s; "
                      f"host has {os.cpu_count()} logical CPUs, BLAS threads {blas}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    import torch
    import synth
    from paper_2204_06204_amd.grid import Grid

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    p = synth.config("cfg3")
    g = Grid.from_problem(p)

    if args.profile_only:
        if args.profile_only == "apply":
            for dtype in (torch.float32, torch.float64):
                apply_timing(g, p, dtype, args.apply_reps, torch)
        elif args.profile_only == "project":
            print(json.dumps(projection_timing(torch)), flush=True)
        elif args.profile_only == "outer":
            outer_loop(g, p, torch.float32, args.steps, args.warmup, torch, true_obj=False, multi=True)
        elif args.profile_only == "fused_large":
            # FP32 Jacobi-PCG solves of 41 steps (40 fused steps each) on the
            # 384x192x192 cantilever with one load case
            import synth as _s
            g.close()
            p = _s.config("cfg5")
            g = Grid.from_problem(p, max_rhs=1)
            dev = torch.device("cuda:0")
            rho = torch.tensor(p.x0, dtype=torch.float32, device=dev)
            f = torch.tensor(p.loads[0], dtype=torch.float32, device=dev)
            u = torch.zeros_like(f)
            for _ in range(args.warmup + args.steps):
                u.zero_()
                g.inner_solve(rho, f, u, 41)
            torch.cuda.synchronize()
        elif args.profile_only == "plane":
            plane_path(torch)
        else:
            outer_loop(g, p, torch.float32, args.steps, args.warmup, torch, krylov=KRYLOV_DEGREE,
                       true_obj=False)
        # a streaming kernel that reads and writes COPY_BYTES (b = 2 a, plain
        # global loads and stores) scales the HBM counters
        a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        print(f"profile-only {args.profile_only} done", flush=True)
        return

    dt32, st32 = outer_loop(g, p, torch.float32, args.steps, args.warmup, torch, multi=True)
    dt32c, _ = outer_loop(g, p, torch.float32, args.steps, args.warmup, torch, true_obj=False)
    steps64 = max(10, args.steps // 2)
    dt64, st64 = outer_loop(g, p, torch.float64, steps64, args.warmup // 2, torch, multi=True)
    steps_cp = max(10, args.steps // 4)
    dtcp, stcp = outer_loop(g, p, torch.float32, steps_cp, args.warmup // 2, torch, krylov=KRYLOV_DEGREE)
    dtcp64, _ = outer_loop(g, p, torch.float64, steps_cp, args.warmup // 2, torch, krylov=KRYLOV_DEGREE,
                           true_obj=False)
    steps_pgd = 10
    dtpgd, stpgd = outer_loop(g, p, torch.float32, steps_pgd, 2, torch, exact_rtol=PGD_RTOL)
    t_apply32 = apply_timing(g, p, torch.float32, args.apply_reps, torch)
    t_apply64 = apply_timing(g, p, torch.float64, args.apply_reps, torch)
    t_apply32_cold = apply_timing(g, p, torch.float32, args.apply_reps, torch, cold=True)
    t_apply64_cold = apply_timing(g, p, torch.float64, args.apply_reps, torch, cold=True)
    t_apply32_bin = apply_timing(g, p, torch.float32, args.apply_reps, torch, binary=True)
    t_fused = fused_step_timing(g, p, torch)

    ndof, E = p.ndof, p.E
    N = ndof // 3
    bytes32 = 2 * ndof * 4 + E * 4          # read u, write y, read one density per element
    bytes64 = 2 * ndof * 8 + E * 8
    # fused CG step: read x, r, p, s, w, D^-1 and write x, r, p, s, w (3N floats
    # each), read the mask byte per node and one density per element
    bytes_fused = 11 * ndof * 4 + N + E * 4
    achieved = bytes_fused / t_fused / 1e9
    traffic = measured_traffic("k_apply<float, 1, 3, false>", "outer_step_pmc.json")
    # algorithmic bytes of one outer iteration (FP32, m inner steps), kernel by kernel
    m = p.inner_steps
    bytes_outer = (2 * E * 4                                    # filter, in the final pass below: 1/Hs in, rho out
                   + 5 * ndof * 4 + N + E * 4                   # residual: u, f in; r, z, D^-1 out
                   + 3 * ndof * 4 + N + E * 4                   # step 0 product: z, r in; w out
                   + (m - 1) * bytes_fused                      # fused steps
                   + 8 * ndof * 4 + N + 3 * E * 4               # last step + sensitivity: x r p s w D^-1 f in, x out; rho, 1/Hs in, g out
                   + 3 * E * 4                                  # filter transpose with the step: g, x in, y out
                   + 2 * E * 4                                  # projection: one or two working passes
                   + 3 * E * 4)                                 # final projection pass: y, x_old in, x out (and the filter's x)

    fixed = None if args.no_fixed_err else fixed_error(g, p, torch)
    sizes = None if args.no_sizes else apply_sizes(torch)
    fsizes = None if args.no_sizes else fused_sizes(torch)
    osizes = None if args.no_sizes else outer_sizes(torch)
    proj = None if args.no_sizes else projection_timing(torch)
    fixed4 = None if (args.no_sizes or args.no_fixed_err) else fixed_error_cfg4(torch)
    hist = None if args.no_sizes else optimality_history(g, p, torch)
    plane = None if args.no_sizes else plane_path(torch)
    cpu = None if args.no_cpu_baseline else cpu_baseline(p, args.cpu_seconds)

    value = args.steps / dt32
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "outer_iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded U[0.2,0.4] densities, unit tip load), no dataset",
        "config": {"workload": "hex8 cantilever 128x64x64 (524,288 elements, 1,635,075 DOFs), "
                               "one outer iteration = filter r=2 + 8 Jacobi-PCG steps + sensitivity "
                               "+ filter^T + mean-projected step + FP64 volume projection; the timed "
                               "iterations run in one fbto_outer_steps call",
                   "elements": E, "dofs": ndof, "inner_steps": p.inner_steps, "volfrac": p.volfrac,
                   "filter_radius": p.filter_radius, "alpha0": ALPHA0_CFG3,
                   "precision": "fp32 storage and arithmetic, fp64 dot products / norms / projection"},
        "apply_K": {
            "fp32_us": t_apply32 * 1e6, "fp32_gdof_s": ndof / t_apply32 / 1e9,
            "fp32_hbm_frac": bytes32 / t_apply32 / 1e9 / HBM_PEAK_GBS,
            "fp32_binary_density_us": t_apply32_bin * 1e6,
            "fp64_us": t_apply64 * 1e6, "fp64_gdof_s": ndof / t_apply64 / 1e9,
            "fp32_cold_us": t_apply32_cold * 1e6, "fp32_cold_gdof_s": ndof / t_apply32_cold / 1e9,
            "fp64_cold_us": t_apply64_cold * 1e6, "fp64_cold_gdof_s": ndof / t_apply64_cold / 1e9,
            "fp64_hbm_frac": bytes64 / t_apply64 / 1e9 / HBM_PEAK_GBS,
            "fp32_cold_hbm_frac": bytes32 / t_apply32_cold / 1e9 / HBM_PEAK_GBS,
            "fp64_cold_hbm_frac": bytes64 / t_apply64_cold / 1e9 / HBM_PEAK_GBS,
        },
        "apply_K_sizes": sizes,
        "one_call_per_iteration": {"outer_iter_s": args.steps / dt32c, "ms_per_step": dt32c / args.steps * 1e3,
                                   "note": "the same FP32 iterations, one fbto_outer_step call each (value: "
                                           "the K timed iterations in one fbto_outer_steps call)"},
        "fp64_path": {"outer_iter_s": steps64 / dt64, "ms_per_step": dt64 / steps64 * 1e3},
        "cpfbto_path": {"outer_iter_s": steps_cp / dtcp, "ms_per_step": dtcp / steps_cp * 1e3,
                        "krylov_degree": KRYLOV_DEGREE, "beta": 1.0, "products_per_step": KRYLOV_DEGREE + 3,
                        "final_state": stcp,
                        "fp64_outer_iter_s": steps_cp / dtcp64,
                        "note": "Alg. 3 (CPFBTO): one low-level step with the Krylov preconditioner of "
                                "Eq. LSP per outer iteration, FP32 (and FP64: fp64_outer_iter_s)"},
        "final_state": {"fp32": st32, "fp64": st64},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_apply<float, 1, CGF> (fused Jacobi-PCG step, 7 of the 8 steps of an "
                               "outer iteration), algorithmic bytes 11*3N*4 + N + E*4 = "
                               f"{bytes_fused} per launch, {t_fused * 1e6:.2f} us per launch"},
        "fused_step_sizes": fsizes,
        "outer_roofline": {"bytes_per_iter": bytes_outer, "ceiling_iter_s": HBM_PEAK_GBS * 1e9 / bytes_outer,
                           "frac": value * bytes_outer / (HBM_PEAK_GBS * 1e9)},
        "pgd_path": {"outer_iter_s": steps_pgd / dtpgd, "ms_per_step": dtpgd / steps_pgd * 1e3,
                     "rtol": PGD_RTOL, "final_state": stpgd,
                     "note": "projected gradient descent with the low-level problem solved to rtol "
                             "(FP32 Jacobi-PCG, warm-started), the paper's baseline"},
        "fixed_error": fixed,
        "fixed_error_cfg4": fixed4,
        "outer_sizes": osizes,
        "projection": proj,
        "optimality_history": hist,
        "plane_path": plane,
        "cpu_baseline": cpu,
        "kernel_hash": kernel_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
