"""Benchmark of the MLSDC-SH hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-graph]
                    [--no-extra] [--only legendre|mixed|adjoint|large|dome] [--dome-hours H]

A step is one two-level MLSDC time step (Algorithm 1 of the paper) on the
headline workload: fine level T255 on the 768 x 384 Gaussian grid with 5
Gauss-Lobatto nodes, coarse level T127 on 384 x 192 with 3 nodes, 2 fine and
2 coarse sweeps per iteration, 4 iterations, dt = 300 s, FP64, on seeded
synthetic fields (spectra with variance ~ (n+1)^-3, max wind 40 m/s, max
|Phi'| = 1 % of the mean geopotential) that stand in for the paper's
R_f = 256 test cases.  Inputs are resident in HBM before timing.

Prints one JSON line with the throughput (steps/s), the roofline of the
dominant kernel (its launch durations measured with HIP events on its own
stream during an instrumented pass over the same steps), the oracle timed on
the host cores, and secondary figures: the paper's 1+1 sweep variant, the
T127/T63 configuration, Legendre GFLOP/s of the 15-field T255 transform pair
and steps/s per working precision with the error against FP64, the adjoint's
seconds per step (T127/T63, 20 checkpointed steps) and the large
T1023/T511 Gauss-Radau configuration per precision.

`--only dome` runs the Gaussian-dome temporal refinement study instead (one
simulated day at T255/T127 per scheme and time step; errors, observed orders,
GPU seconds, observed MLSDC speedups at matched error).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLSDC-SH steps/s and Legendre GFLOP/s at T255, FP64 vs mixed; adjoint s/step"
HBM_PEAK_GBS = 8000.0

FINE = dict(N=255, J=384, I=768, nodes=5)
COARSE = dict(N=127, J=192, I=384, nodes=3)
C1_FINE = dict(N=127, J=192, I=384, nodes=5)
C1_COARSE = dict(N=63, J=96, I=192, nodes=3)
DT = 300.0
NITER, NSWEEP = 4, 2
SEED = 1005
LARGE_DT = 60.0
PRECISIONS = (("fp64", 0), ("fp32", 1), ("bf16x2", 2), ("bf16x3", 3))
# Legendre tables in device memory (suffix "") or regenerated on the fly (no tables)
TABLE_MODES = (("", 0), ("_onthefly", 1))


def kcount(nmax, m, p):
    return (nmax - m - p) // 2 + 1 if nmax - m - p >= 0 else 0


def legendre_bytes(N, F, terms, fourier_pairs):
    """Algorithmic HBM bytes of one Legendre analysis launch with the FP64
    tables: the table values it sums (`terms`, per latitude pair, after the
    polar truncation; read once), the north and south Fourier rows of the
    `fourier_pairs` (m, latitude pair) it reads and the F-field output (each
    touched once).  Both counts come from the plan (shx_plan_analysis_terms)."""
    table = terms * 8
    ext = (N + 1) * (N + 4) // 2
    return table + 2 * fourier_pairs * F * 16 + ext * F * 16, table


def legendre_flops(N, J, F, nmax):
    Jh = J // 2
    rows = sum(kcount(nmax, m, p) for m in range(N + 1) for p in (0, 1))
    return 4.0 * rows * Jh * F


def kernel_source_sha256(path, signature):
    """SHA-256 of one kernel's source text: from its signature line to the
    closing brace of the function (a line holding only '}')."""
    import hashlib
    with open(path) as f:
        src = f.read()
    a = src.index(signature)
    b = src.index("\n}\n", a)
    return hashlib.sha256(src[a:b + 3].encode()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    record, or None when that kernel's source changed since it was taken."""
    rec = os.path.join(ROOT, "profiles", "k_leg_an_T255_traffic.json")
    try:
        with open(rec) as f:
            d = json.load(f)
        if kernel_source_sha256(os.path.join(ROOT, d["source"]), d["kernel_signature"]) != d["kernel_sha256"]:
            return None
        return d["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def make_stepper(pk, fine, coarse, niter, nsweep, residual=False, precision=0, table_mode=0):
    par = pk.swe_params()
    pf = pk.Plan(fine["N"], fine["J"], fine["I"], precision, table_mode)
    lf = pk.Level(pf, par, pk.SDC_GAUSS_LOBATTO, fine["nodes"])
    lc = None
    if coarse:
        pc = pk.Plan(coarse["N"], coarse["J"], coarse["I"], precision, table_mode)
        lc = pk.Level(pc, par, pk.SDC_GAUSS_LOBATTO, coarse["nodes"])
    return pk.Stepper(lf, lc, niter=niter, nsweep_fine=nsweep, nsweep_coarse=nsweep, residual_check=residual)


def run_steps(torch, stepper, x0, steps, warmup, graph, dt=DT):
    """Returns (seconds for `steps` steps, final state)."""
    a = x0.clone()
    b = torch.empty_like(a)
    for _ in range(warmup):
        stepper.step(dt, a, b)
        a, b = b, a
    torch.cuda.synchronize()
    if graph:
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            stepper.step(dt, a, b)           # workspaces exist before capture
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=s):
                stepper.step(dt, a, b)
                # copy back so that each replay advances the state by one step
                a.copy_(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, a
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stepper.step(dt, a, b)
        a, b = b, a
    torch.cuda.synchronize()
    return time.perf_counter() - t0, a


def _median3(fn):
    """Median of 3 timed runs of fn() after one untimed warm-up run (seconds)."""
    fn()
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), ts


def cpu_baseline(state_np, workload):
    """The oracle (plain FP64 torch-CPU, all host threads) on the host cores,
    each figure the median of 3 runs after 1 warm-up: one step of the
    headline T255/T127 workload (the reported value), one T127/T63 step, one
    15-field T255 transform pair, and one T127/T63 adjoint step (forward
    recomputation + reverse pass by torch autograd through the oracle)."""
    import torch
    from oracle import sdc as OS
    from oracle import sht as OH
    from oracle import swe as OW

    def two_level(fine, coarse):
        lf = OS.Level(OW.SWEProblem(fine["N"], fine["J"], fine["I"]), "lobatto", fine["nodes"])
        lc = OS.Level(OW.SWEProblem(coarse["N"], coarse["J"], coarse["I"]), "lobatto", coarse["nodes"])
        R, P = OS.spectral_transfer(fine["N"], coarse["N"])
        return lambda x: OS.mlsdc_step(lf, lc, DT, x, niter=NITER, nsweep_fine=NSWEEP, nsweep_coarse=NSWEEP,
                                       restrict_space=R, interp_space=P)

    step_h = two_level(FINE, COARSE)
    xh = torch.tensor(state_np)
    t_h, ts_h = _median3(lambda: step_h(xh))
    step_c1 = two_level(C1_FINE, C1_COARSE)
    x1 = torch.tensor(workload.state(127, workload.SEEDS["mlsdc_T127"][0]))
    t_c1, _ = _median3(lambda: step_c1(x1))
    g = OH.Grid(FINE["N"], FINE["J"], FINE["I"])
    spec = torch.tensor(workload.states(255, workload.SEEDS["pair_T255"]).reshape(15, -1))
    t_c2, _ = _median3(lambda: g.sh_forward(g.sh_inverse(spec)))
    x3 = torch.tensor(workload.state(127, workload.SEEDS["adjoint_T127"][0]))
    w = torch.where(OH.orders(127) == 0, 1.0, 2.0).to(torch.float64)

    def adjoint_step():
        x = x3.clone().requires_grad_(True)
        y = step_c1(x)
        (0.5 * (w * (y[0].real ** 2 + y[0].imag ** 2)).sum()).backward()
    t_c3, _ = _median3(adjoint_step)
    return {"value": 1.0 / t_h, "unit": "steps/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": "median of 3 runs after 1 warm-up of one step of the same T255/T127 (2,2)x4 workload "
                      f"(plain FP64 torch-CPU oracle; runs {', '.join(f'{t:.1f}' for t in ts_h)} s)",
            "s_per_step_T255_T127": t_h, "s_per_step_T127_T63": t_c1, "s_per_pair_T255_F15": t_c2,
            "s_per_adjoint_step_T127_T63": t_c3}


def variants_extra(pk, torch, workload, x0, steps, graph):
    extra = {}
    # paper's variant: one fine and one coarse sweep per iteration
    st11 = make_stepper(pk, FINE, COARSE, NITER, 1)
    s11, _ = run_steps(torch, st11, x0, max(5, steps // 2), 2, graph)
    extra["steps_per_s_T255_T127_sweeps_1_1"] = max(5, steps // 2) / s11
    # T127/T63 configuration
    x1 = torch.tensor(workload.state(127, 1001), device="cuda")
    stc1 = make_stepper(pk, C1_FINE, C1_COARSE, NITER, NSWEEP)
    s1, _ = run_steps(torch, stc1, x1, max(5, steps), 2, graph)
    extra["steps_per_s_T127_T63_sweeps_2_2"] = max(5, steps) / s1
    # the paper's comparison (Sec. 6): MLSDC(5,3,4,1/2) above vs single-level
    # SDC(5,8) on the fine level alone, same nodes, 8 sweeps
    par = pk.swe_params()
    sdc = pk.Stepper(pk.Level(pk.Plan(FINE["N"], FINE["J"], FINE["I"]), par, pk.SDC_GAUSS_LOBATTO, FINE["nodes"]),
                     None, niter=8, nsweep_fine=1)
    ssdc, _ = run_steps(torch, sdc, x0, max(5, steps // 2), 2, graph)
    sdc_rate = max(5, steps // 2) / ssdc
    extra["steps_per_s_T255_SDC_5_8"] = sdc_rate
    extra["speedup_MLSDC_5_3_4_vs_SDC_5_8"] = extra["steps_per_s_T255_T127_sweeps_1_1"] / sdc_rate
    # three levels (mlsdc_step_multi): T255 / T127 / T63 with 5 / 3 / 2
    # nodes, one sweep per level, 4 iterations, against the two-level
    # (1+1) x 4 step above
    lv3 = [pk.Level(pk.Plan(c["N"], c["J"], c["I"]), par, pk.SDC_GAUSS_LOBATTO, c["nodes"])
           for c in (FINE, COARSE, dict(N=63, J=96, I=192, nodes=2))]
    st3 = pk.MultiStepper(lv3, niter=NITER, nsweeps=1)
    s3, _ = run_steps(torch, st3, x0, max(5, steps // 2), 2, graph)
    extra["steps_per_s_T255_T127_T63_three_levels_1_1_1"] = max(5, steps // 2) / s3
    return extra


def copy_bandwidth(torch, mib=2048):
    """Achievable HBM bandwidth of a plain device copy (read + write bytes / time)."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) * 1e-3 / 10
    del src, dst
    return 2.0 * n * 8 / secs / 1e9


def legendre_extra(pk, torch, workload):
    """Legendre GFLOP/s, T255, 15 fields (one launch per direction), per
    precision, with tables in device memory and without (on the fly)."""
    extra = {}
    spec0 = torch.tensor(workload.states(255, workload.SEEDS["pair_T255"]).reshape(15, -1), device="cuda")
    fl = legendre_flops(255, 384, 15, 255)
    ref_grid = ref_spec = None
    for (pname, prec), (tname, tmode) in ((p, t) for t in TABLE_MODES for p in PRECISIONS):
        plan = pk.Plan(255, 384, 768, prec, tmode)
        spec = spec0.clone()
        grid = plan.inverse(spec)
        spec_b = plan.forward(grid)
        torch.cuda.synchronize()
        if ref_grid is None:
            ref_grid, ref_spec = grid.clone(), spec_b.clone()
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        cin = torch.zeros((256 * 259 // 2) * 15, dtype=torch.complex128, device="cuda")
        four = torch.zeros(384 * 256 * 15, dtype=torch.complex128, device="cuda")
        pk.legendre_synthesis(plan, 15, 255, cin, four)
        e0.record()
        for _ in range(reps):
            pk.legendre_synthesis(plan, 15, 255, cin, four)
        e1.record()
        torch.cuda.synchronize()
        syn_us = e0.elapsed_time(e1) * 1e3 / reps
        e0.record()
        for _ in range(reps):
            pk.legendre_analysis(plan, 15, 255, four, cin)
        e1.record()
        torch.cuda.synchronize()
        an_us = e0.elapsed_time(e1) * 1e3 / reps
        err_g = max((torch.linalg.vector_norm(grid[f] - ref_grid[f]) / torch.linalg.vector_norm(ref_grid[f])).item()
                    for f in range(15))
        err_s = max((torch.linalg.vector_norm(spec_b[f] - ref_spec[f]) / torch.linalg.vector_norm(ref_spec[f])).item()
                    for f in range(15))
        extra[f"legendre_T255_F15_{pname}{tname}"] = {
            "synthesis_gflops": fl / (syn_us * 1e-6) / 1e9, "analysis_gflops": fl / (an_us * 1e-6) / 1e9,
            "synthesis_us": syn_us, "analysis_us": an_us, "flop_per_direction": fl,
            "max_rel_err_vs_fp64_inverse": err_g, "max_rel_err_vs_fp64_roundtrip": err_s,
        }
        del plan
    return extra


def rel_errs(torch, x, ref):
    return [(torch.linalg.vector_norm(x[f] - ref[f]) / torch.linalg.vector_norm(ref[f])).item()
            for f in range(x.shape[0])]


def mixed_steps_extra(pk, torch, x0, steps, graph):
    """The benchmark step with reduced-precision Legendre contractions, with
    tables in device memory and without (on the fly)."""
    extra = {}
    ref_state = None
    n = max(5, steps // 2)
    for (pname, prec), (tname, tmode) in ((p, t) for t in TABLE_MODES for p in PRECISIONS):
        stp = make_stepper(pk, FINE, COARSE, NITER, NSWEEP, precision=prec, table_mode=tmode)
        one = stp.step(DT, x0.clone())
        torch.cuda.synchronize()
        if ref_state is None:
            ref_state = one.clone()
        sp, _ = run_steps(torch, stp, x0, n, 2, graph)
        extra[f"steps_per_s_T255_T127_{pname}{tname}"] = {"value": n / sp,
                                                   "one_step_rel_err_vs_fp64": rel_errs(torch, one, ref_state)}
        del stp
    return extra


def adjoint_extra(pk, torch, workload):
    """T127/T63 levels as in the two-level configuration, 20 steps, per-step
    checkpoints, L = 0.5 ||Phi'(T)||^2, gradient w.r.t. Theta^0."""
    x1 = torch.tensor(workload.state(127, 1003), device="cuda")
    sa = make_stepper(pk, C1_FINE, C1_COARSE, NITER, NSWEEP)
    nadj = 20
    w = torch.ones(x1.shape[1], dtype=torch.float64, device="cuda")
    w[(127 + 1):] = 2.0          # m >= 1 entries follow the (N+1) m = 0 entries
    times = []
    for rep in range(2):
        x = x1.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = pk.integrate(x, sa, DT, nadj)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        (0.5 * (w * (y[0].real ** 2 + y[0].imag ** 2)).sum()).backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    fwd, bwd = times[-1]
    return {"adjoint_T127_T63_20steps": {
        "s_per_step": bwd / nadj, "forward_s_per_step": fwd / nadj,
        "note": "backward = per-step recompute from the checkpoint + reverse sweep, FP64",
        "grad_finite": bool(torch.isfinite(torch.view_as_real(x.grad)).all().item()),
    }}


def large_extra(pk, torch, workload, graph):
    """Fine T1023 (3072 x 1536, 5 Gauss-Radau-right collocation points) over
    coarse T511 (1536 x 768, 3), (2,2) x 4, dt = 60 s, 5 timed steps per
    precision; Legendre tables held in HBM, and regenerated on the fly."""
    x = torch.tensor(workload.state(1023, workload.SEEDS["mlsdc_T1023"][0]), device="cuda")
    par = pk.swe_params()
    extra = {}
    ref = None
    for (pname, prec), (tname, tmode) in ((p, t) for t in TABLE_MODES for p in PRECISIONS):
        lf = pk.Level(pk.Plan(1023, 1536, 3072, prec, tmode), par, pk.SDC_RADAU_RIGHT, 6)
        lc = pk.Level(pk.Plan(511, 768, 1536, prec, tmode), par, pk.SDC_RADAU_RIGHT, 4)
        st = pk.Stepper(lf, lc, niter=NITER, nsweep_fine=NSWEEP, nsweep_coarse=NSWEEP)
        one = st.step(LARGE_DT, x.clone())
        torch.cuda.synchronize()
        if ref is None:
            ref = one.clone()
        secs, _ = run_steps(torch, st, x, 5, 1, graph, dt=LARGE_DT)
        extra[f"steps_per_s_T1023_T511_radau_{pname}{tname}"] = {"value": 5 / secs,
                                                           "one_step_rel_err_vs_fp64": rel_errs(torch, one, ref)}
        del st, lf, lc
    return extra


# Gaussian-dome temporal refinement (Sec. 5.2): schemes as (name, Gauss-
# Lobatto nodes per level from the finest, iterations, truncation per level),
# one sweep per level and iteration (the paper's setting).  Besides the
# paper's schemes: spatial coarsening only (M_f = M_c), temporal coarsening
# only (both levels T255), and a milder spatial coarsening (T170, ratio 2/3).
DOME_SCHEMES = (("SDC(3,4)", (3,), 4, (255,)), ("MLSDC(3,2,2,1/2)", (3, 2), 2, (255, 127)),
                ("SDC(5,8)", (5,), 8, (255,)),
                ("MLSDC(5,3,4,1/2)", (5, 3), 4, (255, 127)), ("MLSDC(5,3,7,1/2)", (5, 3), 7, (255, 127)),
                ("3-level MLSDC(5,3,2;4)", (5, 3, 2), 4, (255, 127, 63)),
                ("MLSDC(3,3,2,1/2)", (3, 3), 2, (255, 127)), ("MLSDC(3,2,2,1)", (3, 2), 2, (255, 255)),
                ("MLSDC(3,2,2,2/3)", (3, 2), 2, (255, 170)))
DOME_PLANS = {255: (255, 384, 768), 170: (170, 256, 512), 127: (127, 192, 384), 63: (63, 96, 192)}
DOME_DTS = (30.0, 60.0, 120.0, 240.0, 480.0, 960.0)
DOME_REF_DT = 15.0


def advance(torch, stepper, x0, dt, nsteps):
    """nsteps steps from x0: the first eager (it also sizes the workspaces),
    the others as replays of a captured one-step graph.  Returns the state
    and the seconds per replayed step."""
    a = x0.clone()
    b = torch.empty_like(a)
    stepper.step(dt, a, b)
    a, b = b, a
    if nsteps == 1:
        torch.cuda.synchronize()
        return a, float("nan")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            stepper.step(dt, a, b)
            a.copy_(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps - 1):
        g.replay()
    torch.cuda.synchronize()
    return a, (time.perf_counter() - t0) / (nsteps - 1)


def degrees(N):
    """Degree n of each coefficient of the m-major spectral layout."""
    return np.concatenate([np.arange(m, N + 1) for m in range(N + 1)])


def dome_extra(pk, torch, workload, t_end=86400.0, dts=DOME_DTS, only=None):
    """Temporal refinement on the Gaussian dome over t_end seconds: L_inf
    errors of the geopotential and vorticity on the fine grid (and the
    area-weighted L2 error of the geopotential) against SDC(5,8) at
    dt = 15 s, observed orders between successive dt, seconds per step, and
    the observed speedup of each MLSDC scheme over its single-level
    counterpart at matched geopotential error (cost of the single-level
    scheme interpolated log-log in its error).  Also the part of the
    reference's geopotential that a coarse level of truncation T_c cannot
    hold (grid maximum of the degrees n > T_c, and the largest coefficient
    magnitude max_m |Phi_n^m| at n = T_c + 1), at t = 0 and t_end, and per
    scheme the grid maximum of the error's degrees n > 127."""
    par = pk.swe_params(phibar=workload.dome_phibar())
    plans = {N: pk.Plan(*v) for N, v in DOME_PLANS.items()}
    pf = plans[255]
    mu, _, wq = pf.latitudes()
    wgt = torch.tensor(wq, device="cuda")[:, None] / (2.0 * FINE["I"])   # area weights, sum 1
    grid = torch.tensor(workload.dome_grid(mu, FINE["I"])[None], device="cuda")
    x0 = torch.zeros(3, workload.nspec(FINE["N"]), dtype=torch.complex128, device="cuda")
    x0[0] = pf.forward(grid)[0]

    def stepper(nodes, k, trunc):
        lv = [pk.Level(plans[t], par, pk.SDC_GAUSS_LOBATTO, n) for t, n in zip(trunc, nodes)]
        return pk.MultiStepper(lv, niter=k, nsweeps=1)

    def fields(x):
        return pf.inverse(x[0:2].contiguous())

    ref, _ = advance(torch, stepper((5,), 8, (255,)), x0, DOME_REF_DT, int(round(t_end / DOME_REF_DT)))
    rg = fields(ref)
    out = {"t_end_s": t_end, "reference": f"SDC(5,8), dt = {DOME_REF_DT:g} s", "dt_s": list(dts),
           "alpha": workload.DOME["alpha"], "schemes": {}, "truncated_part_phi": {}}
    deg = torch.tensor(degrees(FINE["N"]), device="cuda")
    for tc in (127, 170):
        tp = {}
        for tag, x in (("t0", x0), ("t_end", ref)):
            hi = torch.where(deg > tc, x[0], torch.zeros_like(x[0]))
            tp["grid_max_" + tag] = pf.inverse(hi[None].contiguous())[0].abs().max().item()
            tp["max_coef_n%d_" % (tc + 1) + tag] = x[0][deg == tc + 1].abs().max().item()
        out["truncated_part_phi"]["T%d" % tc] = tp
    for name, nodes, k, trunc in DOME_SCHEMES:
        if only and name not in only:
            continue
        errs, errz, err2, cost, errhi = [], [], [], [], []
        st = stepper(nodes, k, trunc)
        for dt in dts:
            x, sps = advance(torch, st, x0, dt, int(round(t_end / dt)))
            d = fields(x) - rg
            dhi = torch.where(deg > 127, x[0] - ref[0], torch.zeros_like(x[0]))
            errhi.append(pf.inverse(dhi[None].contiguous())[0].abs().max().item())
            errs.append(d[0].abs().max().item())
            errz.append(d[1].abs().max().item())
            err2.append(math.sqrt((wgt * d[0] * d[0]).sum().item()))
            cost.append(sps * t_end / dt)
        order = [math.log2(errs[i + 1] / errs[i]) if errs[i] > 0 and errs[i + 1] > 0 else float("nan")
                 for i in range(len(errs) - 1)]
        out["schemes"][name] = {"linf_phi": errs, "linf_zeta": errz, "l2_phi": err2, "order_phi": order,
                                "gpu_seconds": cost, "linf_phi_degrees_above_127": errhi}
        del st
        print(f"# dome {name}: linf_phi {['%.3g' % e for e in errs]}", file=sys.stderr, flush=True)
    for ml, sl in (("MLSDC(3,2,2,1/2)", "SDC(3,4)"), ("MLSDC(5,3,4,1/2)", "SDC(5,8)"),
                   ("3-level MLSDC(5,3,2;4)", "SDC(5,8)"), ("MLSDC(3,2,2,2/3)", "SDC(3,4)")):
        if ml not in out["schemes"] or sl not in out["schemes"]:
            continue
        m, s1 = out["schemes"][ml], out["schemes"][sl]
        for key, tag in (("linf_phi", ""), ("l2_phi", "_l2")):
            pts = [(a, b) for a, b in zip(s1[key], s1["gpu_seconds"]) if a > 0 and math.isfinite(a)]
            le = np.log(np.array([a for a, _ in pts]))
            lc = np.log(np.array([b for _, b in pts]))
            sp = []
            for e, c in zip(m[key], m["gpu_seconds"]):
                ok = len(pts) > 1 and e > 0 and le.min() <= math.log(e) <= le.max()
                if not ok:
                    sp.append(float("nan"))
                    continue
                o = np.argsort(le)
                sp.append(float(np.exp(np.interp(math.log(e), le[o], lc[o])) / c))
            m["speedup" + tag + "_vs_" + sl] = sp
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--only", choices=["legendre", "mixed", "adjoint", "large", "dome"], default=None,
                    help="run only this group of secondary measurements and print them as one JSON line "
                         "(for profiler runs)")
    ap.add_argument("--dome-hours", type=float, default=24.0,
                    help="simulated time of the Gaussian-dome refinement study (--only dome)")
    ap.add_argument("--dome-dts", default=",".join(f"{v:g}" for v in DOME_DTS),
                    help="comma-separated time steps (s) of the Gaussian-dome study")
    ap.add_argument("--dome-schemes", default=None,
                    help="semicolon-separated subset of the Gaussian-dome schemes (default: all)")
    ap.add_argument("--dome-alpha", type=float, default=None,
                    help="dome width parameter alpha in exp(-alpha (d/a)^2) (default: the workload's)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB once (a plain copy kernel of "
                         "known size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the MLSDC-SH path runs on a "
              "single GPU and does not shard across GPUs.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1805_07923_amd as pk
    import workload
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    pk.lib()
    torch.cuda.set_device(0)
    if args.dome_alpha is not None:
        workload.DOME["alpha"] = args.dome_alpha
    state_np = workload.state(FINE["N"], SEED)
    x0 = torch.tensor(state_np, device="cuda")
    if args.only:
        graph = not args.no_graph
        run = {"legendre": lambda: legendre_extra(pk, torch, workload),
               "mixed": lambda: mixed_steps_extra(pk, torch, x0, args.steps, graph),
               "adjoint": lambda: adjoint_extra(pk, torch, workload),
               "large": lambda: large_extra(pk, torch, workload, graph),
               "dome": lambda: dome_extra(pk, torch, workload, args.dome_hours * 3600.0,
                                          tuple(float(v) for v in args.dome_dts.split(",")),
                                          args.dome_schemes.split(";") if args.dome_schemes else None)}[args.only]
        print(json.dumps({"only": args.only, "extra": run()}), flush=True)
        return

    stepper = make_stepper(pk, FINE, COARSE, NITER, NSWEEP)
    graph = not args.no_graph
    secs, xk = run_steps(torch, stepper, x0, args.steps, args.warmup, graph)
    value = args.steps / secs
    finite = bool(torch.isfinite(torch.view_as_real(xk)).all().item())

    # kernel time per step by class (HIP events around each launch of one
    # class, on the launch stream; includes a few us of event overhead each)
    evals_fine = 1 + NITER * NSWEEP * (FINE["nodes"] - 1)
    evals_coarse = 1 + NITER * (COARSE["nodes"] - 1) * (1 + NSWEEP)
    kinds = {}
    for name, kc in (("legendre_analysis", pk.KC_LEGENDRE_AN), ("legendre_synthesis", pk.KC_LEGENDRE_SYN),
                     ("grid_fft_products", pk.KC_GRID), ("sdc_node", pk.KC_SDC_NODE)):
        a = x0.clone()
        b = torch.empty_like(a)
        with pk.KernelTimer(kc, 2 * (evals_fine + evals_coarse) + 16) as kt:
            stepper.step(DT, a, b)
            torch.cuda.synchronize()
        kinds[name] = float(np.sum(kt.ms))

    # dominant kernel: the Legendre analysis of a fine-level tendency (5
    # fields, degrees <= N+1), timed over back-to-back launches of the same
    # kernel in the same launch configuration on the same stream
    pf = stepper.fine.plan
    NF = FINE["N"]
    ne = (NF + 1) * (NF + 4) // 2
    g_in = torch.randn(FINE["J"] * (NF + 1) * 5, dtype=torch.complex128, device="cuda")
    s_out = torch.empty(ne * 5, dtype=torch.complex128, device="cuda")
    for _ in range(5):
        pk.legendre_analysis(pf, 5, NF + 1, g_in, s_out)
    reps = 200
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pk.legendre_analysis(pf, 5, NF + 1, g_in, s_out)
    e1.record()
    torch.cuda.synchronize()
    an_us = e0.elapsed_time(e1) * 1e3 / reps
    terms, fpairs = pf.analysis_terms(FINE["N"] + 1)
    abytes, table_bytes = legendre_bytes(FINE["N"], 5, terms, fpairs)
    achieved = abytes / (an_us * 1e-6) / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * secs / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "two-level MLSDC-SH step: fine T255 on 768x384 Gaussian grid, 5 Gauss-Lobatto nodes; "
                        "coarse T127 on 384x192, 3 nodes; 2 fine + 2 coarse sweeps per iteration, 4 iterations, "
                        "dt=300 s; seeded (n+1)^-3 spectra, max wind 40 m/s, |Phi'| 1% of 2.94e4",
            "fine": "T255 768x384 GL5", "coarse": "T127 384x192 GL3", "niter": NITER,
            "nsweep_fine": NSWEEP, "nsweep_coarse": NSWEEP, "dt_s": DT, "precision": "fp64",
            "hip_graph": graph, "parallelism": "single GPU",
            "evaluations_per_step": {"fine": evals_fine, "coarse": evals_coarse},
        },
        "roofline": {
            "kernel": "k_leg_an (Legendre analysis from the table on the matrix cores, fine level, 5 fields)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
            "avg_launch_us": an_us, "algorithmic_bytes_per_launch": abytes,
            "measured_copy_gbs": copy_bandwidth(torch),
            "table_bytes": table_bytes, "timed_launches": reps,
        },
        "kernel_ms_per_step": kinds,
        "final_state_finite": finite,
    }
    if not args.no_extra:
        extra = {}
        extra.update(variants_extra(pk, torch, workload, x0, args.steps, graph))
        extra.update(legendre_extra(pk, torch, workload))
        extra.update(mixed_steps_extra(pk, torch, x0, args.steps, graph))
        extra.update(adjoint_extra(pk, torch, workload))
        extra.update(large_extra(pk, torch, workload, graph))
        out["extra"] = extra
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": n * 8, "bytes_written": n * 8}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(state_np, workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
