"""Benchmark of the fast gravity / gravity-gradient forward operator.

Workload: the paper-scale grid, nx = ny = 1024, nz = 100, 20 m cubic cells,
stations 10 m above the top, all six components (gz, gxx, gxy, gxz, gyy, gyz);
density = 20 seeded random prisms plus a Gaussian random field.  A step is
one forward apply d = G rho with the kernel spectra resident in HBM and the
density already on the device; the plan (kernel table + spectra) is built
once before the timed region and its time is reported as ``plan_ms``.

Metric: effective kernel evaluations per second, B * C * N_d * N_m / t,
the number of kernel-matrix entries the operator applies per second
(C = 6 components, N_d = nx*ny stations, N_m = nx*ny*nz cells).

One JSON line is printed.  Besides the headline FP64 forward it carries the
FP32 path, the adjoint, a live roofline of the dominant kernel (the column
pass) with the device's practical copy and read rates beside the 8 TB/s
peak, the same model with other component sets (gz with the first
derivatives gx, gy; all nine outputs) and on a depth-stretched layered mesh,
the equal-dimension survey (as many observation levels as layers),
the batched inversion-step workload (512^2 x 128, 32 models, forward
and adjoint in both precisions), the CPU oracle timed on a bounded sample,
and a served-latency run:
a seeded Poisson trace of mixed requests (4000 at 200 req/s by default)
replayed through the FP32 continuous-batching server (p50/p99 latency
overall and apart for requests whose kernel spectra were resident on
arrival and for those that waited for them to be built, and the ten
slowest requests), and its first 3 s through the plain FP64 operator (FIFO,
one model per call).
"""

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "effective N_d·N_m kernel-evals/s at 1024²×100 6-comp; p50/p99 served latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_colpass_paper_scale.json")
KERNEL_SOURCES = ["colpass.hip", "gf_fft.h", "gf_lane.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2005_10160_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def nyquist_chunks(nz):
    """Layer chunks of the real Nyquist column unit (the column pass runs it
    apart from the main units): up to 32 chunks."""
    target = min(nz, 32)
    lps = (nz + target - 1) // target
    return (nz + lps - 1) // lps


def colpass_algorithmic_bytes(p, B):
    """Bytes the forward column pass must move per launch: every resident
    spectrum value once, the row-transformed density columns once, and the
    partial data columns once (per layer split for the main units, per layer
    chunk for the real Nyquist unit; quarter-plane spectra, one real per
    frequency; complex intermediates)."""
    info = p.info
    s = 8 if p.precision == "f64" else 4
    M = info.px // 2            # column units (kx = 0 and Px/2 share unit 0)
    Q = info.py // 2 + 1        # quarter-plane frequencies along y
    spectra = info.n_spec * info.nz * (M + 1) * Q * s
    R = B * info.nz * M * info.ny * 2 * s
    ws = p.workspace_bytes("forward", B)
    S = int((ws // (2 * s * M * info.ny) - B * info.nz) // (B * info.n_spec))
    D = S * B * info.n_spec * M * info.ny * 2 * s
    Dny = nyquist_chunks(info.nz) * B * info.n_spec * info.ny * s
    return spectra + R + D + Dny, S


def settle(fn, seconds=0.3, max_calls=300):
    """Untimed applies for a fraction of a second before the warm-up steps:
    after idle the device runs its first applies up to 25 % slower while its
    clocks ramp (kernel traces show the column pass settling over about
    20 applies), and the timed steps are meant to measure the steady state."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while n < max_calls and time.perf_counter() - t0 < seconds:
        fn()
        n += 1
        if n % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def time_forward(p, rho, d, ws, steps, warmup):
    import torch
    settle(lambda: p.forward(rho, d, ws))
    for _ in range(warmup):
        p.forward(rho, d, ws)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record()
        p.forward(rho, d, ws)
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return per, wall


def time_passes(p, rho, d, ws, steps, op="forward"):
    """Per-pass durations from HIP events recorded by the library on the
    launch stream around each pass."""
    import torch
    p.set_timing(True)
    out = []
    for _ in range(steps):
        if op == "forward":
            p.forward(rho, d, ws)
        else:
            p.adjoint(d, rho, ws)
        out.append(p.last_pass_ms(op))
    p.set_timing(False)
    torch.cuda.synchronize()
    return np.array(out)


def batched_step(steps, warmup):
    """Inversion-step workload: 512 x 512 x 128, 20 m cells, h = 10 m, all six
    components, 32 density models sharing the geometry (uniform(-0.5, 0.5)
    g/cm^3 plus a 4x4x3 +1.0 g/cm^3 block per model, drawn on the device from
    a seeded generator).  One batched forward and one batched adjoint per
    precision, median of `steps` applies after `warmup`."""
    import torch
    import paper_2005_10160_amd as gf
    from synth import PRESETS
    g = PRESETS["inversion"]
    B = 32
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(400)
    out = {"workload": "inversion step, %dx%dx%d, %g m cells, h=%g m, 6 components, batch %d"
                       % (g.nx, g.ny, g.nz, g.dx, g.h, B)}
    evals = float(B) * 6 * g.nd * g.nm
    for prec in ("f32", "f64"):
        dt = torch.float64 if prec == "f64" else torch.float32
        s = 8 if prec == "f64" else 4
        log("bench: batched %s" % prec)
        p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, gf.ALL6, prec, device=dev)
        rho = (torch.rand((B, g.nz, g.ny, g.nx), generator=gen, device=dev, dtype=dt) - 0.5) * 1000.0
        for b in range(B):
            l0, m0, n0 = (int(v) for v in torch.randint(0, g.nx - 4, (3,), generator=gen, device=dev).tolist())
            n0 = 1 + n0 % (g.nz - 4)
            rho[b, n0:n0 + 3, m0:m0 + 4, l0:l0 + 4] += 1000.0
        d = torch.empty((B, 6, g.ny, g.nx), dtype=dt, device=dev)
        gout = torch.empty_like(rho)
        wsb = max(p.workspace_bytes("forward", B), p.workspace_bytes("adjoint", B))
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        res = {}
        for op in ("forward", "adjoint"):
            run = (lambda: p.forward(rho, d, ws)) if op == "forward" else (lambda: p.adjoint(d, gout, ws))
            settle(run)
            for _ in range(warmup):
                run()
            torch.cuda.synchronize()
            times = []
            for _ in range(steps):
                a = torch.cuda.Event(enable_timing=True)
                e = torch.cuda.Event(enable_timing=True)
                a.record()
                run()
                e.record()
                torch.cuda.synchronize()
                times.append(a.elapsed_time(e))
            ms = statistics.median(times)
            # transform and reduction flop at 5 N log2 N per complex transform
            # of N points: the row transforms (a real row of Px values as a
            # complex one of Px/2), one column transform per layer and unit,
            # 4 flop per frequency, layer and component for the reduction,
            # and the inverse transforms per component
            info = p.info
            U = info.px // 2 + 1
            lg = lambda n: math.log2(n)
            rowf = 5 * (info.px // 2) * lg(info.px // 2)
            colf = 5 * info.py * lg(info.py)
            flop = B * (g.nz * g.ny * rowf + g.nz * U * colf + 4 * 6 * g.nz * U * info.py
                        + 6 * U * colf + 6 * g.ny * rowf)
            peak_tf = 78.6 if prec == "f64" else 157.3
            # compulsory bytes: resident spectra once, every model's density
            # (or residual) and data once
            spectra = p.spectra_bytes
            io = B * s * (g.nz * g.nx * g.ny + 6 * g.nx * g.ny)
            res[op] = {"ms": round(ms, 3), "effective_evals_per_s": evals / (ms * 1e-3),
                       "compulsory_GBs": round((spectra + io) / (ms * 1e-3) / 1e9, 1),
                       "compulsory_frac_of_8TBs": round((spectra + io) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
                       "fft_TFLOPs": round(flop / (ms * 1e-3) / 1e12, 2),
                       "fft_frac_of_vector_peak": round(flop / (ms * 1e-3) / 1e12 / peak_tf, 3)}
        out[prec] = res
        p.close()
        del rho, d, gout, ws
        torch.cuda.empty_cache()
    return out


def config_table(dev, rho_c3, steps=20, warmup=3):
    """The per-configuration table: for the tiny (16^2x8), the medium
    (256^2x64) and the paper-scale grid, in FP64 and FP32: median forward and
    adjoint apply times, effective evaluations per second and compulsory
    bytes over the forward time as a fraction of 8 TB/s.  (Errors against
    the oracle come from the tests.)"""
    import torch
    import paper_2005_10160_amd as gf
    from synth import PRESETS, tiny_density, prisms_and_grf

    def median_ms(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return statistics.median(ts)

    out = {}
    for name, g in (("C1_tiny", PRESETS["tiny"]), ("C2_medium", PRESETS["medium"]),
                    ("C3_paper_scale", PRESETS["paper_scale"])):
        log("bench: config table %s" % name)
        if name == "C1_tiny":
            rho = tiny_density(g.nx, g.ny, g.nz)
        elif name == "C2_medium":
            rho = prisms_and_grf(g.nx, g.ny, g.nz, 6, 202, 203)
        else:
            rho = rho_c3
        row = {"grid": "%dx%dx%d" % (g.nx, g.ny, g.nz)}
        for prec in ("f64", "f32"):
            dt = torch.float64 if prec == "f64" else torch.float32
            p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, gf.ALL6, prec, device=dev)
            x = torch.from_numpy(rho).to(dev, dt).unsqueeze(0)
            d = torch.empty((1,) + p.data_shape, dtype=dt, device=dev)
            gt = torch.empty_like(x)
            ws = torch.empty(max(p.workspace_bytes("forward", 1), p.workspace_bytes("adjoint", 1)),
                             dtype=torch.uint8, device=dev)
            tf = median_ms(lambda: p.forward(x, d, ws))
            ta = median_ms(lambda: p.adjoint(d, gt, ws))
            s_el = 8 if prec == "f64" else 4
            comp = p.spectra_bytes + s_el * (g.nz * g.nx * g.ny + 6 * g.nx * g.ny)
            row[prec] = {"forward_ms": round(tf, 4), "adjoint_ms": round(ta, 4),
                         "effective_evals_per_s": 6.0 * g.nd * g.nm / (tf * 1e-3),
                         "compulsory_frac_of_8TBs": round(comp / (tf * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            p.close()
            del x, d, gt, ws
        out[name] = row
    return out


def stream_bandwidth(dev, gib=2, reps=10):
    """Practical streaming rates of the device, timed with HIP events: a
    plain device-to-device copy of `gib` GiB (GB/s of bytes read plus
    written) and a sum over 2*`gib` GiB (read-only, like the column pass)."""
    import torch
    n = (gib << 30) // 8
    src = torch.ones(2 * n, dtype=torch.float64, device=dev)
    dst = torch.empty(n, dtype=torch.float64, device=dev)
    out = torch.empty((), dtype=torch.float64, device=dev)

    def rate(fn, nbytes):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return nbytes / (a.elapsed_time(b) / reps * 1e-3) / 1e9

    copy = rate(lambda: dst.copy_(src[:n]), 2.0 * n * 8)
    read = rate(lambda: torch.sum(src, dim=0, out=out), 2.0 * n * 8)
    del src, dst, out
    return copy, read


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, rho_np, n_stations, threads):
    import oracle
    if threads:
        oracle.set_threads(threads)
    from synth import sample_stations
    st = sample_stations(g.nx, g.ny, 0, seed=1)[[8, 0, 3, 5]][:n_stations]
    t0 = time.perf_counter()
    oracle.forward(g, rho_np, st)
    dt = time.perf_counter() - t0
    evals = len(st) * g.nm * 6
    full = 6.0 * g.nd * g.nm
    # the same direct sum built in plain double, timed beside it
    t0 = time.perf_counter()
    oracle.forward_fp64(g, rho_np, st)
    dt64 = time.perf_counter() - t0
    return {
        "value": evals / dt,
        "unit": "kernel-evals/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": "long-double direct sum (eq. 3) of the same 1024^2x100 model at %d station(s), "
                  "all %d cells, 6 components counted; %.1f s wall" % (len(st), g.nm, dt),
        "cpu": cpu_model(),
        "extrapolated_full_apply_s": full / (evals / dt),
        "fp64_mode": {"value": evals / dt64, "unit": "kernel-evals/s",
                      "sample": "the same stations, plain double arithmetic; %.1f s wall" % dt64},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32 side run")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--cpu-stations", type=int, default=2)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 32-model inversion-step timing")
    ap.add_argument("--no-sets", action="store_true", help="skip the gz/gx/gy and nine-component timings")
    ap.add_argument("--configs", action="store_true",
                    help="add the per-configuration table (tiny, medium, paper scale: apply times)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of the replayed request trace at 200 req/s (0: no serving run)")
    ap.add_argument("--serve-records", default=None,
                    help="write one CSV line per served request (arrival, admission, completion, cache hit)")
    ap.add_argument("--small", action="store_true", help="medium 256^2x64 grid (quick check)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 1 GiB elementwise copy (read 1 GiB, write 1 GiB) so that "
                         "hardware byte counters can be scaled")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the operator runs on a single MI355X and has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2005_10160_amd as gf
    from synth import PRESETS, prisms_and_grf

    g = PRESETS["medium" if args.small else "paper_scale"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("bench: generating density %dx%dx%d" % (g.nx, g.ny, g.nz))
    rho_np = prisms_and_grf(g.nx, g.ny, g.nz, 20 if not args.small else 6, 302, 303)

    def run(prec, steps, warmup, with_adjoint, mask=gf.ALL6, zedges=None, levels=1):
        dt = torch.float64 if prec == "f64" else torch.float32
        log("bench: plan %s, components 0x%x%s%s" % (prec, mask, "" if zedges is None else ", layered",
                                                    "" if levels == 1 else ", %d levels" % levels))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if levels != 1:
            p = gf.plan_levels(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, levels, mask, prec, device=dev)
        elif zedges is None:
            p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, mask, prec, device=dev)
        else:
            p = gf.plan_layered(g.nx, g.ny, g.dx, g.dy, zedges, g.h, mask, prec, device=dev)
        plan_wall = (time.perf_counter() - t0) * 1e3
        rho = torch.from_numpy(rho_np).to(dev, dt)
        d = torch.empty((1,) + p.data_shape, dtype=dt, device=dev)
        wsb = max(p.workspace_bytes("forward", 1), p.workspace_bytes("adjoint", 1))
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        log("bench: timing %s forward" % prec)
        per, wall = time_forward(p, rho.unsqueeze(0), d, ws, steps, warmup)
        passes = time_passes(p, rho.unsqueeze(0), d, ws, steps)
        res = {"plan": p, "per": per, "wall": wall, "passes": passes, "plan_ms": plan_wall,
               "spectra_bytes": p.spectra_bytes, "ws_bytes": wsb}
        if with_adjoint:
            log("bench: timing %s adjoint" % prec)
            g_out = torch.empty((1, g.nz, g.ny, g.nx), dtype=dt, device=dev)
            for _ in range(warmup):
                p.adjoint(d, g_out, ws)
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(steps)]
            for a, e in ev:
                a.record()
                p.adjoint(d, g_out, ws)
                e.record()
            torch.cuda.synchronize()
            res["adjoint_ms"] = statistics.median(a.elapsed_time(e) for a, e in ev)
            res["adjoint_passes"] = time_passes(p, g_out, d, ws, steps, "adjoint")
        return res

    if args.calibrate:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    evals = 6.0 * g.nd * g.nm
    main_res = run(args.precision, args.steps, args.warmup, not args.no_adjoint)
    per = main_res["per"]
    # the apply time is the median of the timed applies
    ms_per_step = statistics.median(per)
    value = evals / (ms_per_step * 1e-3)

    p = main_res["plan"]
    # compulsory bytes of one apply: resident spectra once, density in, data
    # out (the intermediate spectra of the density are not counted)
    s_el = 8 if args.precision == "f64" else 4
    compulsory = (p.spectra_bytes + s_el * (g.nz * g.nx * g.ny + 6 * g.nx * g.ny))
    model_bytes, S = colpass_algorithmic_bytes(p, 1)
    # the dominant kernel's average launch duration, from HIP events the
    # library records on the launch stream around the column pass
    col_ms = float(np.mean(main_res["passes"][:, 1]))
    achieved = compulsory / (col_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE) and not args.small:
        try:
            tr = json.load(open(TRAFFIC_FILE))
            if tr.get("kernel_hash") == kernel_hash() and tr.get("precision") == args.precision:
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "col_forward_ws_kernel (FFT along y + layer reduction + inverse FFT)",
                "kernel_ms": round(col_ms, 4),
                "algorithmic_bytes_per_launch": int(compulsory),
                "algorithmic_bytes": "compulsory bytes of one apply (resident spectra once, density in, "
                                     "data out); one column-pass launch serves one apply",
                # what the kernel itself must move (spectra, the row-transformed
                # density and the partial data columns), and the counters' bytes
                "kernel_model_bytes_per_launch": model_bytes,
                "kernel_model_GBs": round(model_bytes / (col_ms * 1e-3) / 1e9, 1),
                "kernel_model_frac": round(model_bytes / (col_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic_frac": (None if traffic is None
                                 else round(traffic / (col_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)),
                "layer_splits": S}
    pct = np.percentile(per, [10, 50, 90])
    log("bench: device streaming rates")
    copy_gbs, read_gbs = stream_bandwidth(dev)
    roofline["practical_copy_GBs"] = round(copy_gbs, 1)
    roofline["practical_read_GBs"] = round(read_gbs, 1)
    roofline["kernel_model_frac_of_read"] = round(model_bytes / (col_ms * 1e-3) / 1e9 / read_gbs, 4)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "kernel-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "%s forward, %dx%dx%d, %gx%gx%g m cells, h=%g m, 6 components, batch 1"
                               % ("medium" if args.small else "paper-scale", g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h),
                   "nx": g.nx, "ny": g.ny, "nz": g.nz, "components": 6, "batch": 1,
                   "precision": args.precision},
        "roofline": roofline,
        "mean_ms": float(np.mean(per)),
        "p10_ms": float(pct[0]),
        "p90_ms": float(pct[2]),
        "apply_compulsory": {"bytes": int(compulsory),
                             "GBs": round(compulsory / (ms_per_step * 1e-3) / 1e9, 1),
                             "frac_of_8TBs": round(compulsory / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "plan_ms": round(main_res["plan_ms"], 1),
        "spectra_bytes": main_res["spectra_bytes"],
        "pass_ms": [round(float(x), 4) for x in main_res["passes"].mean(axis=0)],
        # stored-kernel counts of the paper (eq. 5 dense, eq. 9 and eq. 11
        # origin kernels, eq. 22 BTTB, eq. 20 ratio) beside the resident bytes
        "storage": p.storage(),
    }
    # the plan again in the warm process: the first plan of a process also
    # pays the device's first large allocations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p2 = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, gf.ALL6, args.precision, device=dev)
    torch.cuda.synchronize()
    line["plan_ms_warm"] = round((time.perf_counter() - t0) * 1e3, 1)
    p2.close()
    del p2
    if "adjoint_ms" in main_res:
        line["adjoint_ms_per_step"] = main_res["adjoint_ms"]
        line["adjoint_pass_ms"] = [round(float(x), 4) for x in main_res["adjoint_passes"].mean(axis=0)]
    p.close()
    del main_res

    if not args.no_f32 and args.precision == "f64":
        r32 = run("f32", args.steps, args.warmup, False)
        ms32 = statistics.median(r32["per"])
        a32, _ = colpass_algorithmic_bytes(r32["plan"], 1)
        c32 = float(np.mean(r32["passes"][:, 1]))
        comp32 = r32["spectra_bytes"] + 4 * (g.nz * g.nx * g.ny + 6 * g.nx * g.ny)
        line["f32"] = {"value": evals / (ms32 * 1e-3), "ms_per_step": ms32,
                       "pass_ms": [round(float(x), 4) for x in r32["passes"].mean(axis=0)],
                       "roofline_frac": round(comp32 / (c32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "apply_compulsory_frac_of_8TBs": round(comp32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "kernel_model_GBs": round(a32 / (c32 * 1e-3) / 1e9, 1),
                       "plan_ms": round(r32["plan_ms"], 1)}
        r32["plan"].close()
        del r32

    if not args.no_sets:
        # other component sets on the same model: the first derivatives with
        # gz, and all nine outputs (eight resident spectra, two column-pass
        # launches of six and two); and the six components on a layered mesh
        # (layers thickening from 5 m by 3 % per layer, 2.4 km deep)
        stretched = [0.0] + list(np.cumsum(5.0 * 1.03 ** np.arange(g.nz)))
        sets = {}
        for name, mask, ze in (("gz_gx_gy", gf.GZ | gf.GX | gf.GY, None), ("all9", gf.ALL9, None),
                               ("layered_all6", gf.ALL6, stretched)):
            sets[name] = {}
            for prec in ("f64", "f32"):
                r = run(prec, 10, 2, True, mask, ze)
                ms = statistics.median(r["per"])
                nout = r["plan"].n_out
                sets[name][prec] = {"components": nout, "ms_per_step": round(ms, 4),
                                    "effective_evals_per_s": nout * g.nd * g.nm / (ms * 1e-3),
                                    "pass_ms": [round(float(x), 4) for x in r["passes"].mean(axis=0)],
                                    "adjoint_ms": round(r["adjoint_ms"], 4),
                                    "plan_ms": round(r["plan_ms"], 1),
                                    "spectra_bytes": r["spectra_bytes"]}
                r["plan"].close()
                del r
        line["component_sets"] = sets

        # the equal-dimension survey: as many observation levels as layers
        # (stations on 100 planes 20 m apart above the model), six
        # components and gz alone; the plan picks how its levels run
        # (reported as level_path: 3 the direct Toeplitz product in depth,
        # 4 the same through the transform in depth)
        lev = {"levels": g.nz, "workload": "equal-dimension survey, %dx%dx%d model, %d observation levels, "
                                           "batch 1" % (g.nx, g.ny, g.nz, g.nz)}
        for name, mask in (("all6", gf.ALL6), ("gz", gf.GZ)):
            lev[name] = {}
            for prec in ("f64", "f32"):
                r = run(prec, 3, 1, True, mask, None, g.nz)
                ms = statistics.median(r["per"])
                evals_l = r["plan"].n_out * g.nz * g.nd * g.nm
                lev[name][prec] = {"ms_per_step": round(ms, 3), "effective_evals_per_s": evals_l / (ms * 1e-3),
                                   "pass_ms": [round(float(x), 3) for x in r["passes"].mean(axis=0)],
                                   "adjoint_ms": round(r["adjoint_ms"], 3),
                                   "adjoint_pass_ms": [round(float(x), 3) for x in r["adjoint_passes"].mean(axis=0)],
                                   "level_path": r["plan"].level_path, "level_chunk": r["plan"].level_chunk,
                                   "plan_ms": round(r["plan_ms"], 1), "spectra_bytes": r["spectra_bytes"]}
                if name == "all6" and prec == "f64":
                    lev["storage"] = r["plan"].storage()
                r["plan"].close()
                del r
        line["levels"] = lev

    if not args.no_batched and not args.small:
        line["batched"] = batched_step(5, 1)

    if args.configs:
        line["configs"] = config_table(dev, rho_np)

    if args.serve_seconds > 0:
        from paper_2005_10160_amd import serve
        line["served"] = serve.bench_served(args.serve_seconds, records_path=args.serve_records)

    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(g, rho_np, args.cpu_stations, args.cpu_threads)

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
