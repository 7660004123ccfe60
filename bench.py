"""Throughput of the split potential solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: one density on a 2048 x 2048 grid over [-16, 16)^2, rho = |u|^2 with
u a seeded sum of 8 anisotropic complex Gaussians (centres in [-6, 6]^2,
widths in [0.5, 2], random phases; seed 0), 64 radial x 128 azimuthal polar
nodes, NUFFT tolerance 1e-7 (FP32 data path) and 1e-12 (FP64 data path).

A step is one potential solve Phi = I1 + I2 (every kernel of the chain) with
rho already resident in device memory.  `value` is FP32 solves/s over K timed
steps, each timed leg preceded by W untimed steps and then by untimed replays
for WARM_SECONDS of wall time (`warmup_s`); the same line carries the FP64 rate, the FP32/FP64 ratio, the rate of
forward + transposed solve pairs, the relative errors of both data paths
against the FP64 oracle, the dominant kernel's ALU and HBM roofline figures (HIP events
recorded around every kernel on its launch stream) and the oracle's own rate
on the host cores.  Further legs (skipped with --no-extra-legs): a batch
of 256 densities with sides drawn from {128, 256, 512, 1024} at h = 1/32
(seed 1; default node sorts), forward + transposed solve pairs at
1024^2 over [-16, 16)^2 (mixture seed 2), 500 split steps of the DS system at
2048^2 with the checkpointed gradient of the final L4 norm, the standard
periodic FFT solver (throughput, and time to accuracy against the split
solver), and the paper's H-E dynamics comparison at 1024^2 (fourth-order
splitting with either potential solver against the exact solution).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Φ solves/s at 2048² grid: FP32 vs FP64 at rel-err 1e-6; fwd+bwd solves/s"
HBM_PEAK_GBS = 8000.0
# Vector ALU peak of MI355X from its unit counts: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops (FMA) x 2.4 GHz = 78.64 TFLOP/s, FP32 and FP64 alike, for code without
# packed FP32 instructions (the kernels are compiled without them).  The published FP32
# figure, 157.3 TFLOP/s, counts packed FP32 (two FMAs per lane).
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
VALU_PEAK_PUBLISHED_F32 = 157.3

# HBM traffic of the dominant kernel (FP32 cols_highfreq, 2048^2) from two rocprofv3
# --pmc passes (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch, mean over the
# dispatches of a short eager run), each scaled by what the same counter reads for
# a plain 256 MiB device copy in the same run.  Valid only for the kernel sources
# whose SHA-256 is recorded: after any change to them `traffic` is reported as null
# until the counters are taken again.
TRAFFIC_RECORD = {
    "kernel": "cols_highfreq",
    "fetch_kib": 16750.6, "write_kib": 32784.0,
    "copy_fetch_kib": 131088.81, "copy_write_kib": 262144.0, "copy_true_kib": 262144.0,
    "sources": ("device_common.hpp", "fft_reg.hpp", "solver_device.hpp", "solver_kernels.hip",
                "solver_kernels.hpp"),
    "sha256": "3d5e1e29587292106d23ea2405c8dc4333448a25899ae7fb8a3465ef031cc42a",
}

N = 2048
HALF = 16.0
N_R, N_THETA = 64, 128
TOL32, TOL64 = 1e-7, 1e-12
SEED = 0


def kernel_bytes(info: dict, real_bytes: int) -> dict:
    """Algorithmic HBM bytes of one launch of each kernel: what the kernel must
    read and write at least (inputs once, outputs once), from the plan's sizes."""
    n, q, m, w = info["n"], info["patch"], info["n_nodes"], info["kernel_width"]
    sr, sc = real_bytes, 2 * real_bytes
    spec = (info["n_fine"] // 2 + 1) * n * sc   # I1 half spectrum, F/2+1 columns of N values
    tiles = info["n_sub"] * info["tile"] ** 2 * sc
    out = {
        "rows_forward": n * n * sr + spec + q * n * sc,
        "cols_highfreq": 2 * spec,
        "cols_type2": q * n * sc + q * q * sc,
        # window, per-node taps (2w), first-tap cell (2 int32) and q_j (FP64); tiles out
        "nodes": q * q * sc + m * (2 * w * sr + 8 + 8) + tiles,
        # tiles and their index lists in, type-1 column transforms out
        "cols_type1": tiles + info["n_contrib"] * 4 + (q * q + 1) * 4 + n * q * sc,
        "rows_inverse": spec + n * q * sc + n * n * sr,
    }
    # the one-stream layout's last launch: the type-1 window columns and every I1 column
    out["type1_highfreq"] = out["cols_type1"] + out["cols_highfreq"]
    return out


def kernel_flops(info: dict) -> dict:
    """Algorithmic flops of one launch of each FFT kernel, by the conventional
    count of 5 F log2 F real flops per complex F-point transform (a count of the
    transform, not of the pruned code, which does less)."""
    n, q, f = info["n"], info["patch"], info["n_fine"]
    fft = 5 * f * math.log2(f)
    out = {"rows_forward": n * fft, "cols_highfreq": 2 * (f // 2 + 1) * fft, "rows_inverse": n * fft,
           "cols_type2": q * fft, "cols_type1": q * fft}
    out["type1_highfreq"] = out["cols_type1"] + out["cols_highfreq"]
    return out


def solve_alg_bytes(n: int, real_bytes: int) -> int:
    """Bytes a solve must move at least: rho in, Phi out, and two passes over the
    half spectrum of the padded transform (N (n_f/2 + 1) complex values) that a
    row-column realisation cannot keep on chip."""
    return 2 * n * n * real_bytes + 4 * n * (n + 1) * 2 * real_bytes


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from TRAFFIC_RECORD, or None when it covers
    another kernel or the kernel sources changed since the counters were taken."""
    import hashlib
    rec = TRAFFIC_RECORD
    if kernel != rec["kernel"]:
        return None
    h = hashlib.sha256()
    for name in rec["sources"]:
        with open(os.path.join(ROOT, "paper_1409_2014_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sha256"]:
        return None
    fetch = rec["fetch_kib"] * rec["copy_true_kib"] / rec["copy_fetch_kib"]
    write = rec["write_kib"] * rec["copy_true_kib"] / rec["copy_write_kib"]
    return round((fetch + write) * 1024)


# Untimed replays before every timed leg, by wall time rather than by count: a
# short timed region (the default --steps of a quick run is a few ms of work)
# otherwise starts before the GPU's clocks have settled, and reads slow.
WARM_SECONDS = 0.3


def warm(fn, torch, seconds: float = WARM_SECONDS) -> None:
    """Run fn until `seconds` of wall time have passed (at least once), then synchronise."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            break


def timed_rate(fn, steps: int, torch) -> float:
    warm(fn, torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def rel_errs(got: np.ndarray, ref: np.ndarray) -> dict:
    return {"rel_linf": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))),
            "rel_l2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}


def cpu_baseline(rho_used: np.ndarray):
    """The FP64 oracle, as it is, on the host cores: one full solve of the same
    2048^2 density (direct nonuniform sums through BLAS, I1 through numpy's FFT)."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
    except ImportError:          # pragma: no cover
        threadpool_info = None
    p = O.SplitParams(n=N, h=2 * HALF / N, n_r=N_R, n_theta=N_THETA)
    # repeat whole solves until about 10 s of host time has been spent
    runs, t0 = 0, time.perf_counter()
    while True:
        ref = O.phi(rho_used, p)
        runs += 1
        if time.perf_counter() - t0 >= 10.0:
            break
    dt = (time.perf_counter() - t0) / runs
    threads = 1
    if threadpool_info is not None:
        blas = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if blas:
            threads = int(max(d.get("num_threads", 1) for d in blas))
    # the small FP64 case (exp(-r^2), 64^2 over [-8, 8)^2, 32 x 64 nodes) on one core
    small = {}
    try:
        from threadpoolctl import threadpool_limits
        import workloads as W
        rho_small = W.gaussian_density(64, 8.0)
        p_small = O.SplitParams(n=64, h=0.25, n_r=32, n_theta=64)
        with threadpool_limits(limits=1):
            O.phi(rho_small, p_small)
            reps, t1 = 0, time.perf_counter()
            while reps < 20 or time.perf_counter() - t1 < 1.0:
                O.phi(rho_small, p_small)
                reps += 1
            small = {"small_64_one_core_ms": round(1e3 * (time.perf_counter() - t1) / reps, 3)}
    except ImportError:          # pragma: no cover
        pass
    return ref, {"value": 1.0 / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
                 "sample": f"{runs} FP64 oracle solve(s) of the same 2048^2 density, {dt:.2f} s each ("
                           f"{len(os.sched_getaffinity(0))} host cores visible)", **small}


def time_split(kernels: dict) -> dict:
    fft = sum(kernels[k]["avg_us"] for k in ("rows_forward", "cols_highfreq", "rows_inverse") if k in kernels)
    node = sum(kernels[k]["avg_us"] for k in ("cols_type2", "nodes", "cols_type1") if k in kernels)
    return {"fft_side_us": round(fft, 2), "node_side_us": round(node, 2),
            "node_side_fraction": round(node / (fft + node), 3) if fft + node > 0 else None,
            "node_side_concurrent": True}


def capture_graph(fn, torch):
    """One captured graph per step kind; a timed step is one replay (the graph
    holds exactly the kernels of one call of fn)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    return graph.replay


def event_kernels(timed_call, steps: int, nbytes: dict) -> dict:
    """Average duration of each kernel over `steps` runs of timed_call (HIP
    events recorded on each kernel's launch stream) and its algorithmic GB/s."""
    acc: dict[str, float] = {}
    for _ in range(steps):
        for name, ms in timed_call():
            acc[name] = acc.get(name, 0.0) + ms
    out = {}
    for name, tot in acc.items():
        ms = tot / steps
        b = nbytes.get(name)
        out[name] = {"avg_us": round(ms * 1e3, 2), "alg_bytes": b,
                     "gbs": round(b / (ms * 1e-3) / 1e9, 1) if b else None}
    return out


def batch_leg(args, torch, ps, W) -> dict:
    """256 independent densities with sides drawn from {128, 256, 512, 1024} at
    h = 1/32 (seed 1), FP32, the default node sort (bin 4, 64 nodes per
    subproblem: under graph replay it beat the plan-time autotuner's picks,
    2.27 against 2.39 ms per batch), one launch per stage over all
    members (the node-side launches on a second stream beside the I1
    columns), replayed from a captured graph."""
    members = W.batch_members(seed=1, count=256)
    params = [dict(n=n, h=2 * half / n, n_r=N_R, n_theta=N_THETA, tol=TOL32)
              for n, half, _ in members]
    print("[bench] batch: planning and building 256 densities", file=sys.stderr, flush=True)
    bp = ps.BatchPlan(params, dtype=torch.float32)
    packed = bp.pack([W.mixture_density(n, half, spec) for n, half, spec in members])
    out = torch.empty_like(packed)

    def fn():
        bp.solve(packed, out)

    for _ in range(max(2, args.warmup // 4)):
        fn()
    if args.launch == "graph":
        fn = capture_graph(fn, torch)
        fn()
    k = max(10, args.steps // 10)
    t = timed_rate(fn, k, torch)
    step_s = t / k
    alg = sum(solve_alg_bytes(n, 4) for n, _, _ in members)
    # algorithmic bytes of each batched launch: the members' single-solve figures summed
    nbytes = {"rows_forward": 0, "cols_type2": 0, "cols": 0, "nodes": 0, "cols_type1": 0, "rows_inverse": 0}
    sizes = {}
    for i, (n, _, _) in enumerate(members):
        info = bp.member_info(i)
        kb = kernel_bytes(info, 4)
        for name in ("rows_forward", "cols_type2", "nodes", "cols_type1", "rows_inverse"):
            nbytes[name] += kb[name]
        nbytes["cols"] += kb["cols_highfreq"]
        if n not in sizes:
            sizes[n] = {"members": 0, "bin": info["bin"], "sub_nodes": info["sub_nodes"]}
        sizes[n]["members"] += 1
    kernels = event_kernels(lambda: bp.solve_timed(packed, out), 3, nbytes)
    res = {"members": len(members), "points": int(bp.total), "solves_per_s": len(members) / step_s,
           "ms_per_step": 1e3 * step_s, "alg_bytes": alg,
           "alg_gbs": round(alg / step_s / 1e9, 1), "roofline_frac": round(alg / step_s / 1e9 / HBM_PEAK_GBS, 4),
           "kernels": kernels, "sizes": {str(n): v for n, v in sorted(sizes.items())}, "steps": k}
    bp.close()
    return res


def adjoint_leg(args, torch, ps, W) -> dict:
    """Forward + transposed solve pairs at 1024^2 over [-16, 16)^2 (mixture seed 2),
    the differentiation workload, both data paths."""
    n, half = 1024, 16.0
    rho = W.mixture_density(n, half, W.draw_mixture(2))
    res = {}
    for name, dt, tol, rb in (("f32", torch.float32, TOL32, 4), ("f64", torch.float64, TOL64, 8)):
        plan = ps.Plan(n, 2 * half / n, dtype=dt, n_r=N_R, n_theta=N_THETA, tol=tol)
        r = torch.as_tensor(rho, dtype=dt, device="cuda")
        o = torch.empty_like(r)
        b = torch.empty_like(r)

        def pair():
            plan.solve(r, o)
            plan.solve_adjoint(o, b)

        for _ in range(args.warmup):
            pair()
        fn = capture_graph(pair, torch) if args.launch == "graph" else pair
        fn()
        k = args.steps
        t = timed_rate(fn, k, torch)
        alg = 2 * solve_alg_bytes(n, rb)
        res[name] = {"pairs_per_s": k / t, "alg_gbs": round(alg * k / t / 1e9, 1),
                     "roofline_frac": round(alg * k / t / 1e9 / HBM_PEAK_GBS, 4)}
        plan.close()
    return res


def stepper_leg(args, torch, ps, W) -> dict:
    """500 Strang steps of the DS system (alpha = beta = 1, tau = 1e-3) on a
    2048^2 grid over [-32, 32)^2 from u0 = exp(-(x^2 + 2 y^2)), one potential
    solve per step; then the gradient of h^2 sum |u(T)|^4 with respect to u0 by
    the reverse pass with a checkpoint every 50 steps.  Both data paths."""
    n, half, steps, every = 2048, 32.0, 500, 50
    x, y, h = W.grid_2d(n, half)
    u0 = np.exp(-(x ** 2 + 2 * y ** 2))
    res = {}
    for name, dt, cdt, tol in (("c64", torch.float32, torch.complex64, TOL32),
                               ("c128", torch.float64, torch.complex128, TOL64)):
        print(f"[bench] stepper {name}: {steps} steps, gradient with checkpoints every {every}",
              file=sys.stderr, flush=True)
        st = ps.DSStepper(n, h, alpha=1.0, beta=1.0, tau=1e-3, dtype=dt, n_r=N_R, n_theta=N_THETA, tol=tol)
        u = torch.as_tensor(u0, dtype=cdt, device="cuda").contiguous()
        w = u.clone()
        st.forward(w, 2)
        st.loss_and_grad(u, 4, 2)
        torch.cuda.synchronize()
        w = u.clone()
        t0 = time.perf_counter()
        st.forward(w, steps)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        m = st.moments(u).cpu().numpy()
        m_end = st.moments(w).cpu().numpy()
        t0 = time.perf_counter()
        loss, g, counts = st.loss_and_grad(u, steps, every)
        torch.cuda.synchronize()
        t_fb = time.perf_counter() - t0
        solves = counts["forward_solves"] + counts["recomputed_solves"] + counts["adjoint_solves"]
        res[name] = {"forward_ms": round(1e3 * t_fwd, 2), "steps_per_s": round(steps / t_fwd, 1),
                     "fwd_bwd_ms": round(1e3 * t_fb, 2), "counts": counts,
                     "fwd_bwd_solves_per_s": round(solves / t_fb, 1),
                     "mass_drift": float(abs(m_end[0] - m[0]) / m[0]), "loss": float(loss),
                     "grad_norm": float(torch.linalg.vector_norm(g))}
        st.close()
        del w, g
    return res


def example1_exact(x, y):
    """Sec. 3.1, Example 1: the potential of rho = pi e^{-pi^2 r^2} in closed form,
    pi [-e^{-q}/2 + (x^2 - y^2) (1 - (1 + q) e^{-q}) / (2 pi^2 r^4)], q = pi^2 r^2,
    and -pi/2 at the origin.  On the grids timed here every other point has
    r >= 1/16, so q >= 0.038 and the bracket loses under 1e-13 to cancellation."""
    r2 = x * x + y * y
    q = math.pi ** 2 * r2
    bracket = -np.expm1(-q) - q * np.exp(-q)
    with np.errstate(invalid="ignore", divide="ignore"):
        aniso = np.where(r2 > 0.0, (x * x - y * y) * bracket / (2.0 * math.pi ** 2 * r2 * r2), 0.0)
    return math.pi * (-0.5 * np.exp(-q) + aniso)


def periodic_leg(args, torch, ps, W) -> dict:
    """The standard periodic FFT solver (the paper's baseline): solves/s on the C2
    density at 2048^2 (both data paths, graph replay), and the paper's
    time-to-accuracy comparison on Example 1 (rho = pi e^{-pi^2 r^2}): the periodic
    solver on [-32, 32)^2 at h = 1/16 against the split solver on [-8, 8)^2 at
    h = 1/4, FP64, errors against the closed form."""
    res = {}
    rho = W.mixture_density(N, HALF, W.draw_mixture(SEED))
    for name, dt in (("f32", torch.float32), ("f64", torch.float64)):
        plan = ps.Plan(N, 2 * HALF / N, dtype=dt, n_r=N_R, n_theta=N_THETA)
        r = torch.as_tensor(rho, dtype=dt, device="cuda")
        o = torch.empty_like(r)

        def fn():
            plan.periodic(r, o)

        for _ in range(args.warmup):
            fn()
        g = capture_graph(fn, torch) if args.launch == "graph" else fn
        g()
        t = timed_rate(g, args.steps, torch)
        res[f"solves_per_s_{name}"] = args.steps / t
        plan.close()

    def example1(half, h, split):
        n = int(round(2 * half / h))
        x, y, _ = W.grid_2d(n, half)
        exact = example1_exact(x, y)
        plan = ps.Plan(n, h, dtype=torch.float64, n_r=N_R, n_theta=N_THETA, tol=TOL64)
        r = torch.as_tensor(W.paper_gaussian_density(n, half), dtype=torch.float64, device="cuda")
        o = torch.empty_like(r)

        def fn():
            (plan.solve if split else plan.periodic)(r, o)

        for _ in range(args.warmup):
            fn()
        g = capture_graph(fn, torch) if args.launch == "graph" else fn
        g()
        t = timed_rate(g, args.steps, torch)
        err = float(np.max(np.abs(o.cpu().numpy() - exact)) / np.max(np.abs(exact)))
        plan.close()
        return {"grid": n, "half_width": half, "h": h, "rel_linf": err, "us_per_solve": round(1e6 * t / args.steps, 2)}

    res["example1_accuracy"] = {"periodic_L32_h1_16": example1(32.0, 1 / 16, False),
                                "split_L8_h1_4": example1(8.0, 0.25, True),
                                "split_L8_h1_8": example1(8.0, 0.125, True)}
    return res


def dynamics_leg(args, torch, ps, W) -> dict:
    """The paper's H-E case I (Sec. 3.2, Tables 7-8): Arkadiev's exact solution of
    the DS system with alpha = 1, beta = -1 on [-64, 64)^2 at h = 1/8 (1024^2),
    400 fourth-order split steps (dt = 0.001, 3 potential solves per step) with
    the potential from the split solver and from the standard periodic FFT
    solver: wall time and relative l2 errors of u and Phi at T = 0.4."""
    half, h, steps, tau = 64.0, 0.125, 400, 1e-3
    n = int(round(2 * half / h))
    x, y, _ = W.grid_2d(n, half)

    def lump(t):
        return 2 * np.exp(1j * (2 * y + 4 * t)) / ((x + 1) ** 2 + (y + 4 * t) ** 2 + 1)

    s_end = (x + 1) ** 2 + (y + 4 * 0.4) ** 2 + 1
    phi_exact = -2 * ((y + 4 * 0.4) ** 2 - x * (x + 2)) / s_end ** 2
    res = {}
    for pot in ("split", "periodic"):
        st = ps.DSStepper(n, h, alpha=1.0, beta=-1.0, tau=tau, dtype=torch.float64, scheme="yoshida4",
                          potential=pot, n_r=N_R, n_theta=N_THETA, tol=TOL64)
        u0 = torch.as_tensor(lump(0.0), dtype=torch.complex128, device="cuda").contiguous()
        w = u0.clone()
        st.forward(w, 3)
        torch.cuda.synchronize()
        u = u0.clone()
        t0 = time.perf_counter()
        st.forward(u, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rho = (u.real ** 2 + u.imag ** 2).contiguous()
        plan = ps.Plan(n, h, dtype=torch.float64, n_r=N_R, n_theta=N_THETA, tol=TOL64)
        phi = (plan.solve(rho) if pot == "split" else plan.periodic(rho)).cpu().numpy()
        un = u.cpu().numpy()
        res[pot] = {"ms_for_400_steps": round(1e3 * dt, 2), "solves": 3 * steps,
                    "rel_l2_u": float(np.linalg.norm(un - lump(0.4)) / np.linalg.norm(lump(0.4))),
                    "rel_l2_phi": float(np.linalg.norm(phi - phi_exact) / np.linalg.norm(phi_exact))}
        st.close()
        plan.close()
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (and the error figures that need it)")
    ap.add_argument("--legs", default="batch,adjoint,stepper,periodic,dynamics",
                    help="comma-separated further legs to run after the 2048^2 single solve "
                         "(batch, adjoint, stepper, periodic, dynamics; empty for none)")
    ap.add_argument("--no-extra-legs", action="store_true", help="same as --legs ''")
    ap.add_argument("--launch", choices=("graph", "eager"), default="graph",
                    help="replay each solve from a captured HIP graph (default) or launch it eagerly")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (a known-size reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solve runs on one GPU "
              "and is not sharded across GPUs", file=sys.stderr)
        return 2

    import torch
    import workloads as W
    import paper_1409_2014_amd as ps

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    h = 2 * HALF / N
    print(f"[bench] building the {N}x{N} density (seed {SEED})", file=sys.stderr, flush=True)
    rho64 = W.mixture_density(N, HALF, W.draw_mixture(SEED))
    rho32_dev = torch.as_tensor(rho64, dtype=torch.float32, device=dev)
    # both data paths see the same (FP32-rounded) input, so one oracle run serves both
    rho_used = rho32_dev.double().cpu().numpy()
    rho64_dev = torch.as_tensor(rho_used, dtype=torch.float64, device=dev)

    plan32 = ps.Plan(N, h, dtype=torch.float32, n_r=N_R, n_theta=N_THETA, tol=TOL32)
    plan64 = ps.Plan(N, h, dtype=torch.float64, n_r=N_R, n_theta=N_THETA, tol=TOL64)
    # the same solve with the node-side chain as separate launches on a second
    # stream (bit-identical results): its per-kernel times split the work by stage
    plan32s = ps.Plan(N, h, dtype=torch.float32, n_r=N_R, n_theta=N_THETA, tol=TOL32, two_streams=True)
    out32 = torch.empty_like(rho32_dev)
    out64 = torch.empty_like(rho64_dev)
    back32 = torch.empty_like(rho32_dev)
    back64 = torch.empty_like(rho64_dev)

    def fwd32():
        plan32.solve(rho32_dev, out32)

    def fwd64():
        plan64.solve(rho64_dev, out64)

    def pair32():
        plan32.solve(rho32_dev, out32)
        plan32.solve_adjoint(out32, back32)

    def pair64():
        plan64.solve(rho64_dev, out64)
        plan64.solve_adjoint(out64, back64)

    def fwd32s():
        plan32s.solve(rho32_dev, out32)

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for fn in (fwd32, fwd64, pair32, pair64, fwd32s):
        for _ in range(args.warmup):
            fn()
    torch.cuda.synchronize()

    if args.launch == "graph":
        fwd32, fwd64, pair32, pair64, fwd32s = (capture_graph(f, torch)
                                                for f in (fwd32, fwd64, pair32, pair64, fwd32s))
        for fn in (fwd32, fwd64, pair32, pair64, fwd32s):
            for _ in range(args.warmup):
                fn()
        torch.cuda.synchronize()

    k = args.steps
    print(f"[bench] timing {k} steps per leg", file=sys.stderr, flush=True)
    t32 = timed_rate(fwd32, k, torch)
    t64 = timed_rate(fwd64, k, torch)
    tp32 = timed_rate(pair32, k, torch)
    tp64 = timed_rate(pair64, k, torch)
    t32s = timed_rate(fwd32s, k, torch)
    phi32 = out32.double().cpu().numpy()
    phi64 = out64.double().cpu().numpy()

    # per-kernel durations from HIP events on each kernel's launch stream, FP32 data path
    print("[bench] per-kernel event timing", file=sys.stderr, flush=True)
    nbytes = kernel_bytes(plan32.info, 4)
    kernels = event_kernels(lambda: plan32.solve_timed(rho32_dev, out32), k, nbytes)
    kernels_split = event_kernels(lambda: plan32s.solve_timed(rho32_dev, out32), k, nbytes)
    # the roofline object covers the longest of the transform kernels (the ones with a
    # flop count); under a profiler's counter passes a node-side kernel can be the
    # longest launch, and it has no flop roof
    flops32 = kernel_flops(plan32.info)
    dominant = max((name for name in kernels if name in flops32), key=lambda name: kernels[name]["avg_us"])
    achieved = kernels[dominant]["gbs"]
    for name, kv in kernels.items():
        if name in flops32:
            kv["tflops"] = round(flops32[name] / (kv["avg_us"] * 1e-6) / 1e12, 2)
    alu_achieved = round(flops32[dominant] / (kernels[dominant]["avg_us"] * 1e-6) / 1e12, 2)
    alg32, alg64 = solve_alg_bytes(N, 4), solve_alg_bytes(N, 8)

    result = {
        "metric": METRIC,
        "value": k / t32,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": k,
        "warmup": args.warmup,
        "warmup_s": WARM_SECONDS,
        "ms_per_step": 1e3 * t32 / k,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single potential solve, 2048x2048 grid over [-16,16)^2, 8-Gaussian mixture "
                               "density (seed 0), 64x128 polar nodes, NUFFT tol 1e-7 (f32) / 1e-12 (f64)",
                   "grid": N, "half_width": HALF, "n_r": N_R, "n_theta": N_THETA,
                   "tol_f32": TOL32, "tol_f64": TOL64, "launch": args.launch},
        "fp64_solves_per_s": k / t64,
        "fp32_over_fp64": t64 / t32,
        "fwd_bwd_solves_per_s": {"f32": k / tp32, "f64": k / tp64},
        "solve_alg_bytes": {"f32": alg32, "f64": alg64},
        "solve_roofline_frac": {"f32": round(alg32 * k / t32 / 1e9 / HBM_PEAK_GBS, 4),
                                "f64": round(alg64 * k / t64 / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_f32": kernels,
        # the two-stream layout: the node-side chain as its own launches beside the I1
        # columns (same results), graph-replayed rate and per-kernel event times
        "two_streams_f32": {"solves_per_s": k / t32s, "kernels": kernels_split},
        # the paper's split of solve time (Sec. 3): FFT-side kernels (I1, with the type-2
        # row transform and the recombination fused in) against the node-side kernels
        "time_split_f32": time_split(kernels_split),
        "node_sort": {"bin": plan32.info["bin"], "sub_nodes": plan32.info["sub_nodes"],
                      "n_sub": plan32.info["n_sub"]},
        # the FFT kernels are bound by their vector ALU work (the counters show
        # 1.0x their algorithmic HBM bytes at a fifth of the bandwidth, and the
        # VALU busy for half the time): the roofline is the ALU one, with the
        # HBM figure of the same kernel beside it
        "roofline": {"bound": "alu", "kernel": dominant, "achieved": alu_achieved,
                     "peak": round(VALU_PEAK_TFLOPS, 2), "unit": "TFLOP/s",
                     "frac": round(alu_achieved / VALU_PEAK_TFLOPS, 4),
                     "traffic": recorded_traffic(dominant),
                     "flops_per_launch": flops32[dominant],
                     "published_peak": VALU_PEAK_PUBLISHED_F32,
                     "frac_of_published": round(alu_achieved / VALU_PEAK_PUBLISHED_F32, 4),
                     "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4)}},
    }
    plan32.close()
    plan64.close()
    plan32s.close()
    legs = set() if args.no_extra_legs else {x.strip() for x in args.legs.split(",") if x.strip()}
    unknown = legs - {"batch", "adjoint", "stepper", "periodic", "dynamics"}
    if unknown:
        print(f"unknown legs {sorted(unknown)}", file=sys.stderr)
        return 2
    if "batch" in legs:
        result["batch_uneven_f32"] = batch_leg(args, torch, ps, W)
    if "adjoint" in legs:
        print("[bench] adjoint pairs at 1024^2", file=sys.stderr, flush=True)
        result["adjoint_pairs_1024"] = adjoint_leg(args, torch, ps, W)
    if "stepper" in legs:
        result["ds_stepper_2048"] = stepper_leg(args, torch, ps, W)
    if "periodic" in legs:
        print("[bench] periodic FFT solver", file=sys.stderr, flush=True)
        result["periodic_fft"] = periodic_leg(args, torch, ps, W)
    if "dynamics" in legs:
        print("[bench] H-E dynamics at 1024^2", file=sys.stderr, flush=True)
        result["he_case1_dynamics_1024"] = dynamics_leg(args, torch, ps, W)
    if not args.no_cpu_baseline:
        print("[bench] oracle leg on the host cores", file=sys.stderr, flush=True)
        ref, base = cpu_baseline(rho_used)
        result["cpu_baseline"] = base
        result["rel_err_vs_oracle"] = {"f32": rel_errs(phi32, ref), "f64": rel_errs(phi64, ref)}
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
