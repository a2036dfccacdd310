#!/usr/bin/env python3
"""Benchmark of the biharmonic-extension solve on one MI355X.

Default workload: the serving stream.  Extension requests arrive as a Poisson
process and are served by the continuous-batching engine (FP64
preconditioner, tol 1e-8): square grids with sides log-uniform in
[128, 2048], Neumann or periodic, multi-circle or star interfaces, F a sum
of 8 Fourier modes, each request distinct and built from its own seed.  The
arrival rate is 0.8 x the saturated rate, measured first on other requests
of the same stream submitted all at once.  The value is completed solves
per second over the timed stream, with p50/p99 latency from arrival to
completion.  Inputs are materialised in device memory before a stream
starts (not counted in latency).  A "step" of this workload is one request:
the timed stream holds max(--steps, --requests) requests.

Beside it (unless --no-extra): the same stream served with the FP32
preconditioner; the 1024^2 star (one solve per step, FP64 at tol 1e-8 and in
accurate mode at tol 1e-13); the 256-instance batch (FP64 and FP32 batched
against one call per instance); the 2048^2 periodic multi-circle case with
the FP32 and FP64 preconditioners; Example 2 (256^3) and Example 4 (1536 x
512, direct and PCG); and the CPU oracle timed on a bounded sample of the
stream.

Other workloads (--workload): star_inward_1024, circle_64,
periodic_circles_2048(_fp64), batch256, example2_256, example4_channel.

Prints ONE JSON line (last line of stdout).  Progress goes to stderr.  Its
`roofline` is the HBM view of the dominant pass (algorithmic bytes per launch
over the launch's time); for the serving stream,
`roofline.column_pass_compute_view` gives the same launches' FP64 flop rate
against the vector peak, since chirp-z cores put the column pass above the
FP64 ridge.
"""
import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "extension solves/sec + p50/p99 latency at 1e-8 rel. residual; HBM GB/s"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
PASS_NAMES = ["stencil", "row_forward", "column", "row_inverse"]
PASS_KERNELS = ["k_stencil", "k_rowfwd", "k_col", "k_rowinv"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from paper_1704_08897_amd import workloads as W
    if name == "star_inward_1024":
        return W.star_inward_problem(1024, tol=1e-8), 0
    if name == "circle_64":
        return W.circle_problem(64, tol=1e-10), 0
    if name == "periodic_circles_2048":
        return W.periodic_circles_problem(2048, tol=1e-8), 1
    if name == "periodic_circles_2048_fp64":
        return W.periodic_circles_problem(2048, tol=1e-8), 0
    raise SystemExit(f"unknown workload {name}")


def pass_coeffs(p, prec):
    """Algorithmic HBM bytes of one launch of pass p for one instance, as
    (bytes per unknown node, bytes per node): each vector read or written
    once, values only at unknown nodes for the CG vectors (loads and stores
    are predicated on the mask), the 1-byte mask where a pass reads it, the
    transform buffer over the whole grid (8 B float64 or 4 B float32)."""
    tb = 8 if prec == 0 else 4
    if p == 0:      # z, p_old read; p_new, q written; mask
        return 32, 1
    if p == 1:      # F, p, q, r read; F, r written; mask; t written
        return 48, 1 + tb
    if p == 2:      # t read and written
        return 0, 2 * tb
    if p == 3:      # t read, r read, z written, mask
        return 16, 1 + tb
    raise ValueError(p)


def column_pass_flops(n):
    """Algorithmic FP64 flops of one 2-D column-pass launch over an n x n grid
    with a Neumann or periodic y axis, by the usual count of 5 m log2(m) per
    complex FFT of m points: the n columns go two to a complex row; each row
    runs a forward and an inverse transform, each one m-point FFT (m = n, a
    power of two) or two through the chirp-z core (m = the power of two at
    least 2n - 1)."""
    import math
    pow2 = n & (n - 1) == 0
    m = n if pow2 else 1 << (2 * n - 2).bit_length()
    ffts = 2 if pow2 else 4
    return (n + 1) // 2 * ffts * 5 * m * math.log2(m)


def pass_bytes(p, n_unknown, N, prec):
    cu, cn = pass_coeffs(p, prec)
    return cu * n_unknown + cn * N


def kernel_source_hash():
    src = os.path.join(ROOT, "paper_1704_08897_amd", "csrc", "bhx_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def load_traffic(kernel, wl):
    """HBM bytes per launch measured by rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, scaled by a copy kernel's reading), from the committed
    summary; None if absent or if the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{wl}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_info():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def percentiles(lat):
    import numpy as np
    a = np.asarray(lat)
    return {"p50": round(1e3 * float(np.median(a)), 2),
            "p99": round(1e3 * float(np.percentile(a, 99)), 2),
            "max": round(1e3 * float(a.max()), 2)}


# ---------------------------------------------------------------------------
# serving stream (default)
# ---------------------------------------------------------------------------

def bench_serve(args):
    """FP64 serving: warm-up, saturated rate, timed Poisson stream; FP32
    served the same way; one profiled stream for the roofline."""
    import numpy as np
    import torch
    from paper_1704_08897_amd import bhx, workloads as W
    from paper_1704_08897_amd.server import Request, Server, serve_stream
    dev = torch.device("cuda:0")
    specs = W.request_stream(10000, seed=5)
    n_timed = max(args.steps, args.requests)
    n_warm = min(8, max(1, args.warmup) * 4)
    a0, a1 = n_warm, n_warm + args.sat_requests
    sets = {"warm": specs[:a0], "sat": specs[a0:a1], "timed": specs[a1:a1 + n_timed]}

    def materialise(ss):
        out = [s.materialise_torch(dev) for s in ss]
        torch.cuda.synchronize()
        return out

    def requests(ss, fields, arrivals):
        return [Request(phi, F, W.bc_code(s.bc, s.bc), 1.0 / s.n, s.tol, arrival=a, tag=s)
                for s, (phi, F), a in zip(ss, fields, arrivals)]

    def progress(tag):
        count = [0]
        t_start = time.perf_counter()

        def on_done(r):
            count[0] += 1
            if count[0] % 20 == 0:
                log(f"{tag}: {count[0]} done, {time.perf_counter() - t_start:.1f} s")
        return on_done

    def run(srv, ss, fields, arrivals, tag):
        reqs = requests(ss, fields, arrivals)
        t0 = time.perf_counter()
        res = serve_stream(srv, reqs, on_done=progress(tag))
        span = max(r.t_done for r in res) - t0
        ok = [r for r in res if r.stats["status"] == bhx.OK]
        return res, ok, span

    def serve(precision, profile=0, timed=True, n_sat=None, n_timed=None):
        srv = Server(0, hbm_budget=args.budget_gb << 30, max_slots=args.slots,
                     precision=precision, profile=profile)
        out = {}
        ns = n_sat or len(sets["sat"])
        nt = n_timed or len(sets["timed"])
        try:
            res_warm, _, _ = run(srv, sets["warm"], fields["warm"], [0.0] * len(sets["warm"]),
                                 "warm-up")
            res, ok, span = run(srv, sets["sat"][:ns], fields["sat"][:ns], [0.0] * ns,
                                f"saturated fp{64 if precision == 0 else 32}")
            sat = len(ok) / span
            out["saturated_solves_per_s"] = round(sat, 3)
            out["saturated_requests"] = ns
            out["saturated_latency_ms"] = percentiles([r.latency for r in res])
            out["saturated_not_converged"] = len(res) - len(ok)
            log(f"saturated (prec {precision}): {sat:.3f} solves/s over {len(res)} requests")
            if profile:
                out["profile"] = bhx.engine_profile(srv.engine)
                # the engine's profile covers the warm-up requests too
                out["served"] = [(r.request.tag.n, r.stats["iterations"])
                                 for r in res_warm + res]
                return out
            if timed:
                rate = 0.8 * sat
                arr = W.poisson_arrivals(nt, rate, seed=6)
                res, ok, span = run(srv, sets["timed"][:nt], fields["timed"][:nt],
                                    list(arr - arr[0]), f"poisson fp{64 if precision == 0 else 32}")
                lat = [r.latency for r in res]
                its = [r.stats["iterations"] for r in res]
                out.update({"solves_per_s": round(len(ok) / span, 3), "requests": len(res),
                            "span_s": round(span, 3), "rate_per_s": round(rate, 3),
                            "latency_ms": percentiles(lat),
                            "iterations": {"mean": round(float(np.mean(its)), 1),
                                           "max": int(max(its))},
                            "not_converged": len(res) - len(ok),
                            "saturation_requests": ns,
                            "sides": [min(s.n for s in sets["timed"][:nt]),
                                      max(s.n for s in sets["timed"][:nt])]})
                log(f"poisson (prec {precision}): {out['solves_per_s']} solves/s, "
                    f"p50 {out['latency_ms']['p50']} ms, p99 {out['latency_ms']['p99']} ms, "
                    f"not converged {out['not_converged']}")
        finally:
            srv.close()
        return out

    t0 = time.perf_counter()
    fields = {k: materialise(v) for k, v in sets.items()}
    log(f"serve: {sum(len(v) for v in sets.values())} distinct requests materialised on the "
        f"device in {time.perf_counter() - t0:.1f} s")
    fp64 = serve(0)
    # the FP32 preconditioner needs 3-4x the iterations: its saturated rate on
    # the first requests of the same phase (all arrive at once)
    fp32 = serve(1, n_sat=8, timed=False) if not args.no_extra else None
    # roofline: the first requests of the saturated phase again, with
    # dispatch events on every pass
    n_prof = min(8, len(sets["sat"]))
    prof_out = serve(0, profile=15, timed=False, n_sat=n_prof)
    prof = prof_out["profile"]
    tot = [prof["ms"][p] for p in range(4)]
    dom = int(np.argmax(tot))
    cu, cn = pass_coeffs(dom, 0)
    launches = prof["launches"][dom]
    alg_total = cu * prof["unknown_nodes"][dom] + cn * prof["nodes"][dom]
    avg_ms = prof["ms"][dom] / max(1, launches)
    alg = alg_total / max(1, launches)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(PASS_KERNELS[dom], "serve"),
                "kernel": PASS_KERNELS[dom], "avg_launch_ms": round(avg_ms, 5),
                "launches": launches, "alg_bytes_per_launch": round(alg),
                "pass_ms_per_launch": {PASS_NAMES[p]: round(prof["ms"][p] /
                                                            max(1, prof["launches"][p]), 5)
                                       for p in range(4)},
                "timed_with": "dispatch start/stop events (hipExtLaunchKernelGGL) on every "
                              "launch of the engine's chunks while a fresh engine serves the "
                              f"warm-up requests and the first {n_prof} requests of the "
                              "saturated phase again; bytes per launch summed over the "
                              "requests each launch worked on"}
    log(f"roofline: {PASS_KERNELS[dom]} {achieved:.1f} GB/s ({achieved / HBM_PEAK_GBS:.3f})")
    # the column pass seen from the arithmetic side: chirp-z cores give it more
    # flops per byte than the FP64 vector ridge (peak flops / peak bandwidth)
    col_ms = prof["ms"][2]
    col_flops = sum(it * column_pass_flops(n) for n, it in prof_out["served"])
    col_bytes = 2 * 8 * prof["nodes"][2]
    if col_ms > 0 and col_bytes > 0:
        tflops = col_flops / (col_ms * 1e-3) / 1e12
        roofline["column_pass_compute_view"] = {
            "bound": "alu", "achieved": round(tflops, 2), "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4),
            "intensity_flop_per_byte": round(col_flops / col_bytes, 1),
            "ridge_flop_per_byte": round(FP64_VECTOR_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9), 1),
            "count": "5 m log2(m) flops per complex m-point FFT; per pair of columns a forward "
                     "and an inverse transform, two FFTs each through a chirp-z core (m the "
                     "power of two >= 2n - 1), one each for a power-of-two side (m = n); "
                     "summed over the profiled requests' iterations"}
        log(f"column pass: {tflops:.2f} TFLOP/s FP64, {col_flops / col_bytes:.1f} flop/B")
    out = {
        "metric": METRIC, "value": fp64["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": fp64["requests"], "warmup": len(sets["warm"]),
        "ms_per_step": round(1e3 * fp64["span_s"] / fp64["requests"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic: seeded serving requests built on the device from their seeds",
        "config": {"workload": "serve_stream", "requests": fp64["requests"],
                   "stream": f"request_stream(seed=5) entries {a1}..{a1 + n_timed - 1}",
                   "side_range": [128, 2048], "bc": "neumann or periodic (1/2 each)",
                   "interfaces": "1-20 circles or star (1/2 each), known inside",
                   "tol": 1e-8, "arrivals": "poisson (seed 6)",
                   "rate_per_s": fp64["rate_per_s"],
                   "saturated_solves_per_s": fp64["saturated_solves_per_s"],
                   "saturation_requests": len(sets["sat"]),
                   "slots": args.slots, "hbm_budget_gb": args.budget_gb,
                   "preconditioner": "fp64", "parallelism": "single_gpu",
                   "latency": "arrival to completion (host monotonic clock); inputs "
                              "materialised in HBM before the stream starts"},
        "latency_ms": fp64["latency_ms"],
        "iterations": fp64["iterations"],
        "not_converged": fp64["not_converged"],
        "roofline": roofline,
    }
    if fp32:
        out["fp32_preconditioner_served"] = fp32
    return out, sets


def cpu_baseline_serve(sets, budget_s):
    """The oracle on the first requests of the timed stream with side <= 384,
    in stream order, until `budget_s` seconds of CPU time (a bounded sample:
    one 2048^2 request takes the oracle many minutes)."""
    import oracle as O
    t_cpu, n, sides = 0.0, 0, []
    for s in sets["timed"]:
        if s.n > 384:
            continue
        p = s.materialise()
        t0 = time.perf_counter()
        O.extend_direct(p.phi, p.F, p.bcx, p.bcy)
        t_cpu += time.perf_counter() - t0
        n += 1
        sides.append(s.n)
        if t_cpu >= budget_s:
            break
    return {"value": round(n / t_cpu, 3), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {n} requests of the timed stream with side <= 384 (sides "
                      f"{min(sides)}-{max(sides)}), one SuperLU factorisation (single-threaded) "
                      "+ 2 long-double refinement steps each; larger requests cost the oracle "
                      "roughly n^3 more", **host_info()}


# ---------------------------------------------------------------------------
# single instance
# ---------------------------------------------------------------------------

def bench_single(p, prec, args, handle, wl, extra=True):
    """Graph-launched solves of one instance; per-pass event timing; the
    dominant kernel's roofline."""
    import numpy as np
    import torch
    from paper_1704_08897_amd import bhx
    N = p.nx * p.ny
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(p.phi).to(dev)
    F = torch.from_numpy(p.F.copy()).to(dev)
    stream = torch.cuda.current_stream()

    def solve(profile=0, tol=None, **kw):
        o = bhx.default_opts(precision=prec, profile=profile, **kw)
        s, st = bhx.extend_ex(handle, phi, F, bc=p.bc, h=p.h, tol=tol or p.tol, opts=o,
                              stream=stream)
        if s != bhx.OK:
            raise SystemExit(f"solve failed: {bhx.status_string(s)} {bhx.last_error()} "
                             f"{st.as_dict()}")
        return st

    for _ in range(args.warmup):
        solve()
    br = solve(profile=15)
    per_pass = [br.pass_ms[k] / max(1, br.pass_launches[k]) for k in range(4)]
    dom = int(np.argmax([br.pass_ms[k] for k in range(4)]))
    log(f"{wl}: pass breakdown (ms/launch): " +
        ", ".join(f"{PASS_NAMES[k]}={per_pass[k]:.4f}" for k in range(4)) +
        f"; iterations={br.iterations}")
    steps = args.steps
    lat, iters = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        st = solve()
        lat.append(time.perf_counter() - ts)
        iters.append(st.iterations)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = steps / elapsed
    log(f"{wl}: {steps} solves in {elapsed:.3f} s -> {value:.2f} solves/s")
    dom_ms, dom_launches = 0.0, 0
    tp0 = time.perf_counter()
    for _ in range(steps):
        stp = solve(profile=1 << dom)
        dom_ms += stp.pass_ms[dom]
        dom_launches += stp.pass_launches[dom]
    torch.cuda.synchronize()
    prof_rate = steps / (time.perf_counter() - tp0)
    avg_ms = dom_ms / max(1, dom_launches)
    alg = pass_bytes(dom, st.n_unknown, N, prec)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    iter_bytes = sum(pass_bytes(k, st.n_unknown, N, prec) for k in range(4))
    iter_ms = sum(per_pass)
    res = {
        "solves_per_s": round(value, 3), "steps": steps,
        "ms_per_solve": round(1e3 * elapsed / steps, 3),
        "latency_ms": {"p50": round(1e3 * statistics.median(lat), 3),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 3)},
        "config": {"nx": p.nx, "ny": p.ny,
                   "bc": ["neumann", "periodic", "dirichlet"][p.bcx] + "x" +
                         ["neumann", "periodic", "dirichlet"][p.bcy],
                   "tol": p.tol, "preconditioner": "fp32" if prec else "fp64",
                   "n_unknown": st.n_unknown},
        "iterations": iters[0], "true_rel_residual": st.true_rel_residual,
        "pass_ms_per_launch": {PASS_NAMES[k]: round(per_pass[k], 5) for k in range(4)},
        "iteration_hbm_gbs": round(iter_bytes / (iter_ms * 1e-3) / 1e9, 1) if iter_ms else None,
        "working_set_mb": round((5 * 8 * st.n_unknown + N * (1 + (8 if prec == 0 else 4)))
                                / 1e6, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(PASS_KERNELS[dom], wl),
                     "kernel": PASS_KERNELS[dom], "avg_launch_ms": round(avg_ms, 5),
                     "launches": dom_launches, "alg_bytes_per_launch": alg,
                     "timed_with": "dispatch start/stop events (hipExtLaunchKernelGGL) on "
                                   f"every launch over {steps} solves (direct launches, "
                                   f"{prof_rate:.2f} solves/s)"},
    }
    if extra and wl == "star_inward_1024":
        # accurate mode at the FP64 bar (tol 1e-13), unpreconditioned CG, direct
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            sta = solve(tol=1e-13, accurate=1, tol_inner=1e-8)
            times.append(time.perf_counter() - ts)
        res["accurate_mode_tol_1e-13"] = {
            "ms_per_solve": round(1e3 * statistics.median(times), 3),
            "iterations": sta.iterations, "restarts": sta.restarts,
            "true_rel_residual": sta.true_rel_residual}
        res["accurate_field"] = F.cpu().numpy()
        ts = time.perf_counter()
        o = bhx.default_opts(precision=0, precond=0, maxit=400000)
        s, stc = bhx.extend_ex(handle, phi, F, bc=p.bc, h=p.h, tol=p.tol, opts=o, stream=stream)
        tc = time.perf_counter() - ts
        res["unpreconditioned_cg"] = {"status": s, "iterations": stc.iterations,
                                      "seconds": round(tc, 3),
                                      "true_rel_residual": stc.true_rel_residual}
        res["direct"] = bench_direct(p, phi, F, handle, stream, bhx)
        res["warm_start_time_step"] = bench_time_step(p, phi, F, handle, stream, bhx)
    solve()                                     # leave F holding the PCG result
    torch.cuda.synchronize()
    res["field"] = F.cpu().numpy()
    del phi, F
    return res


def bench_batch(args, handle, steps):
    """256 uneven instances per step (one batched call, autotuned schedule).
    FP64 batched, the FP32-preconditioner form (standard PCG) and the plain
    FP64 PCG solving the same instances one call each."""
    import numpy as np
    import torch
    from paper_1704_08897_amd import bhx, workloads as W
    probs = W.star_cubic_batch(256, seed=4, tol=1e-8)
    dev = torch.device("cuda:0")
    phis = [torch.from_numpy(p.phi).to(dev) for p in probs]
    Fs = [torch.from_numpy(p.F.copy()).to(dev) for p in probs]
    hs = [p.h for p in probs]
    bcs = [p.bc for p in probs]
    tols = [p.tol for p in probs]
    Ntot = sum(p.nx * p.ny for p in probs)
    stream = torch.cuda.current_stream()

    def run(prec, profile=0, autotune=1):
        o = bhx.default_opts(precision=prec, autotune=autotune, profile=profile)
        s, sts = bhx.extend_batched(handle, phis, Fs, hs, bcs, tols, opts=o, stream=stream)
        if s < 0:
            raise SystemExit(f"batched solve failed: {bhx.status_string(s)} {bhx.last_error()}")
        return sts

    def timed(prec, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            sts = run(prec)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, sts

    t0 = time.perf_counter()
    run(0)
    log(f"batch256: autotune + first FP64 batched solve {time.perf_counter() - t0:.2f} s")
    el, sts = timed(0, steps)
    value = len(probs) * steps / el
    iters = [s.iterations for s in sts]
    br = run(0, profile=15)
    per_pass = [br[0].pass_ms[k] / max(1, br[0].pass_launches[k]) for k in range(4)]
    dom = int(np.argmax([br[0].pass_ms[k] for k in range(4)]))
    alg = sum(pass_bytes(dom, s.n_unknown, p.nx * p.ny, 0) for s, p in zip(br, probs))
    avg_ms = per_pass[dom]
    achieved = alg / (avg_ms * 1e-3) / 1e9
    run(1)
    el32, st32 = timed(1, 1)
    v32 = len(probs) / el32
    o = bhx.default_opts(precision=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it64 = []
    for i in range(len(probs)):
        s, st = bhx.extend_ex(handle, phis[i], Fs[i], bc=bcs[i], h=hs[i], tol=tols[i], opts=o,
                              stream=stream)
        it64.append(st.iterations)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log(f"batch256: FP64 batched {value:.1f}, FP32 batched {v32:.1f}, plain FP64 per instance "
        f"{len(probs) / t_plain:.1f} solves/s")
    return {
        "solves_per_s": round(value, 2), "steps": steps, "instances": len(probs), "nodes": Ntot,
        "ms_per_batch": round(1e3 * el / steps, 3),
        "config": {"side_range": [64, 512], "bc": "mixed neumann/periodic per axis",
                   "tol": 1e-8, "preconditioner": "fp64", "autotune": 1},
        "iterations": {"min": min(iters), "max": max(iters), "mean": float(np.mean(iters))},
        "max_true_rel_residual": max(s.true_rel_residual for s in sts),
        "not_converged": sum(1 for s in sts if s.status != 0),
        "pass_ms_per_launch_first_iterations": {PASS_NAMES[k]: round(per_pass[k], 5)
                                                for k in range(4)},
        "fp32_preconditioner_batched": {
            "solves_per_s": round(v32, 2),
            "mean_iterations": float(np.mean([s.iterations for s in st32])),
            "not_converged": sum(1 for s in st32 if s.status != 0)},
        "plain_fp64_per_instance": {"solves_per_s": round(len(probs) / t_plain, 2),
                                    "mean_iterations": float(np.mean(it64))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "kernel": PASS_KERNELS[dom], "avg_launch_ms": round(avg_ms, 5),
                     "alg_bytes_per_launch": alg,
                     "note": "average over the launches of one profiled batched solve, as "
                             "instances retire"},
    }


def bench_direct(p, phi, F, handle, stream, bhx, reps=3):
    """The same solve by the sparse direct path (banded Cholesky of A_UU on
    the GPU, refined to the same tolerance), and three fields on the same
    phi sharing one factorisation."""
    import torch
    o = bhx.default_opts(solver=1)
    times = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, st = bhx.extend_ex(handle, phi, F, bc=p.bc, h=p.h, tol=p.tol, opts=o, stream=stream)
        times.append(time.perf_counter() - t0)
        if s != bhx.OK:
            raise SystemExit(f"direct solve failed: {bhx.status_string(s)} {bhx.last_error()}")
    sec = statistics.median(times[1:])
    G = [F.clone() for _ in range(3)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s, sts = bhx.extend_fields(handle, phi, G, h=p.h, bc=p.bc, tol=p.tol, opts=o, stream=stream)
    tf = time.perf_counter() - t0
    log(f"direct: {sec * 1e3:.1f} ms per solve; 3 fields {tf * 1e3:.1f} ms")
    return {"ms_per_solve": round(1e3 * sec, 3), "refinement_solves": st.iterations,
            "true_rel_residual": st.true_rel_residual, "three_fields_ms": round(1e3 * tf, 3),
            "method": "banded Cholesky of A_UU (unknowns numbered line by line, here row by row), "
                      "FP64, refined with the compensated residual"}


def bench_time_step(p, phi, F, handle, stream, bhx, reps=3):
    """A level-set time step: the known values move by a smooth 1 % of their
    range; the new extension is solved from zero and from the previous
    extension (warm start), same tolerance."""
    import numpy as np
    import torch
    o = bhx.default_opts()
    bhx.extend_ex(handle, phi, F, bc=p.bc, h=p.h, tol=p.tol, opts=o, stream=stream)
    torch.cuda.synchronize()
    prev = F.cpu().numpy()
    jj, ii = np.meshgrid(np.arange(p.ny) / p.ny, np.arange(p.nx) / p.nx, indexing="ij")
    F1 = p.F + 0.01 * np.abs(p.F).max() * np.sin(2 * np.pi * ii) * np.cos(np.pi * jj)
    known = p.phi < 0
    res = {}
    for name, start, warm in (("cold", F1, 0), ("warm", np.where(known, F1, prev), 1)):
        src = torch.from_numpy(np.ascontiguousarray(start)).to(F.device)
        ow = bhx.default_opts(warm_start=warm)
        times, its = [], []
        for _ in range(reps + 1):
            F.copy_(src)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s, st = bhx.extend_ex(handle, phi, F, bc=p.bc, h=p.h, tol=p.tol, opts=ow,
                                  stream=stream)
            times.append(time.perf_counter() - t0)
            its.append(st.iterations)
        res[name] = {"iterations": its[-1], "ms": round(1e3 * statistics.median(times[1:]), 3)}
    F.copy_(torch.from_numpy(np.ascontiguousarray(p.F)).to(F.device))
    torch.cuda.synchronize()
    res["speedup"] = round(res["cold"]["ms"] / res["warm"]["ms"], 3)
    return res


def bench_periodic(handle, reps=1):
    """The 2048^2 periodic multi-circle case, one solve each with the FP32
    preconditioner (its stated precision) and the FP64 one, tol 1e-8."""
    import torch
    from paper_1704_08897_amd import bhx, workloads as W
    p = W.periodic_circles_problem(2048, tol=1e-8)
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(p.phi).to(dev)
    F = torch.from_numpy(p.F.copy()).to(dev)
    out = {"nx": 2048, "ny": 2048, "bc": "periodic x periodic", "tol": 1e-8,
           "n_unknown": int((p.phi >= 0).sum())}
    for name, prec in (("fp32_preconditioner", 1), ("fp64_preconditioner", 0)):
        o = bhx.default_opts(precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, st = bhx.extend_ex(handle, phi, F, bc=p.bc, h=p.h, tol=p.tol, opts=o)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[name] = {"status": s, "seconds": round(sec, 3), "solves_per_s": round(1 / sec, 4),
                     "iterations": st.iterations, "true_rel_residual": st.true_rel_residual}
        log(f"periodic 2048 prec {prec}: {st.iterations} iterations, {sec:.2f} s")
    del phi, F
    torch.cuda.empty_cache()
    return out


def bench_example2(handle, bhx, n=256, reps=3):
    """Example 2 of the paper at its largest grid (256^3, periodic, tol 1e-6)."""
    import torch
    from paper_1704_08897_amd import workloads as W
    p = W.peanut3d_problem(n)
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(p.phi).to(dev)
    F = torch.from_numpy(p.F.copy()).to(dev)
    times = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, st = bhx.extend3d(handle, phi, F, h=p.h, bc=p.bc, tol=p.tol)
        times.append(time.perf_counter() - t0)
        if s != bhx.OK:
            raise SystemExit(f"3-D solve failed: {bhx.status_string(s)} {st.as_dict()}")
    sec = statistics.median(times[1:])
    log(f"example 2 {n}^3: {st.iterations} iterations, {sec:.3f} s")
    del phi, F
    torch.cuda.empty_cache()
    return {"grid": f"{n}^3", "bc": "periodic^3", "tol": p.tol, "iterations": st.iterations,
            "seconds": round(sec, 4), "true_rel_residual": st.true_rel_residual}


def bench_channel(handle, bhx, ny=512, reps=3):
    """Example 4 of the paper at its largest grid (3 ny x ny = 1536 x 512,
    Neumann sides, periodic top and bottom, ten-term front, tol 1e-6): the
    sparse direct path (unknowns numbered along columns) and PCG."""
    import torch
    from paper_1704_08897_amd import workloads as W
    p = W.channel_problem(ny, terms=10, bcy=W.PERIODIC, tol=1e-6)
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(p.phi).to(dev)
    out = {"grid": f"{3 * ny}x{ny}", "bc": "neumann x periodic", "tol": p.tol,
           "n_unknown": int((p.phi >= 0).sum())}
    for name, solver in (("direct", 1), ("pcg", 0)):
        times = []
        for _ in range(reps + 1):
            F = torch.from_numpy(p.F.copy()).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s, st = bhx.extend_ex(handle, phi, F, bc=p.bc, h=p.h, tol=p.tol,
                                  opts=bhx.default_opts(solver=solver))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            if s != bhx.OK:
                raise SystemExit(f"channel solve failed: {bhx.status_string(s)} {st.as_dict()}")
        out[name] = {"ms_per_solve": round(1e3 * statistics.median(times[1:]), 3),
                     "iterations": st.iterations, "true_rel_residual": st.true_rel_residual}
        log(f"example 4 {3 * ny}x{ny} {name}: {out[name]['ms_per_solve']:.1f} ms, "
            f"{st.iterations} iterations")
    del phi
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="serve")
    ap.add_argument("--requests", type=int, default=48,
                    help="serve: requests in the timed stream (at least --steps)")
    ap.add_argument("--sat-requests", type=int, default=24,
                    help="serve: requests of the saturated phase that sets the arrival rate")
    ap.add_argument("--slots", type=int, default=64, help="serve: engine slots")
    ap.add_argument("--budget-gb", type=int, default=64, help="serve: engine HBM budget")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU time budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the workload itself (no FP32 serving, no other configurations)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "how the path would shard is described in the design notes, not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_08897_amd import bhx

    if args.calib_copy_mb > 0:
        nb = args.calib_copy_mb * (1 << 20)
        a = torch.empty(nb // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log(f"calibration copy: {args.calib_copy_mb} MiB read + written")

    handle = bhx.Handle(0)
    try:
        if args.workload == "serve":
            out, sets = bench_serve(args)
            if not args.no_extra:
                p, _ = workload("star_inward_1024")
                star = bench_single(p, 0, argparse.Namespace(steps=min(args.steps, 10),
                                                             warmup=1), handle,
                                    "star_inward_1024")
                star_field = star.pop("field")
                acc_field = star.pop("accurate_field")
                out["star_inward_1024"] = star
                out["batch256"] = bench_batch(args, handle, steps=2)
                out["periodic_circles_2048"] = bench_periodic(handle)
                out["example2_3d"] = bench_example2(handle, bhx)
                out["example4_channel"] = bench_channel(handle, bhx)
            if not args.no_cpu_baseline:
                import oracle as O
                out["cpu_baseline"] = cpu_baseline_serve(sets, args.cpu_seconds)
                log(f"cpu baseline: {out['cpu_baseline']}")
                if not args.no_extra:
                    # the 1024^2 star's results against the oracle (FP64 bar)
                    t0 = time.perf_counter()
                    ref, _ = O.extend_direct(p.phi, p.F, p.bcx, p.bcy)
                    out["star_inward_1024"]["rel_l2_vs_oracle"] = O.relative_l2(star_field, ref)
                    out["star_inward_1024"]["accurate_mode_tol_1e-13"]["rel_l2_vs_oracle"] = \
                        O.relative_l2(acc_field, ref)
                    out["star_inward_1024"]["cpu_oracle_seconds"] = round(
                        time.perf_counter() - t0, 3)
        elif args.workload == "batch256":
            out = bench_batch(args, handle, steps=args.steps)
            out.update({"metric": METRIC, "value": out["solves_per_s"], "unit": "solves/s",
                        "n_gpus": 1, "warmup": 1, "dtype": "f64", "data": "synthetic",
                        "higher_is_better": True, "scaling": "weak", "vs_baseline": None})
        elif args.workload == "example2_256":
            out = {"workload": "example2_256", **bench_example2(handle, bhx)}
        elif args.workload == "example4_channel":
            out = {"workload": "example4_channel", **bench_channel(handle, bhx)}
        else:
            p, prec = workload(args.workload)
            res = bench_single(p, prec, args, handle, args.workload, extra=not args.no_extra)
            field = res.pop("field")
            res.pop("accurate_field", None)
            out = {"metric": METRIC, "value": res["solves_per_s"], "unit": "solves/s",
                   "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                   "ms_per_step": res["ms_per_solve"], "higher_is_better": True,
                   "scaling": "weak", "vs_baseline": None,
                   "dtype": "f64" if prec == 0 else "f64+f32", "data": "synthetic",
                   "config": {"workload": args.workload, **res.pop("config"),
                              "parallelism": "single_gpu"}, **res}
            if not args.no_cpu_baseline:
                import oracle as O
                t = []
                for _ in range(2):
                    t0 = time.perf_counter()
                    ref, _ = O.extend_direct(p.phi, p.F, p.bcx, p.bcy)
                    t.append(time.perf_counter() - t0)
                out["cpu_baseline"] = {"value": round(len(t) / sum(t), 4), "unit": "solves/s",
                                       "cores": 1, "kind": "oracle",
                                       "sample": f"{len(t)} complete oracle solves of this "
                                                 "workload", **host_info()}
                out["rel_l2_vs_oracle"] = O.relative_l2(field, ref)
    finally:
        handle.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
