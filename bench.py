"""Throughput benchmark of the coupled lattice update (one GPU).

Workload: the bubble ensemble -- a 4096 x 4096 periodic D2Q9 lattice with 200
gas bubbles (radii uniform in [10, 60], non-overlapping, seed 0) in liquid,
density ratio 1000, viscosity ratio 100, gravity from Eo = 10 at Re = 35,
W = 4, SF-11 filter, K = 2 velocity sweeps.  A step is one whole coupled
update of every node (gather, three FD stages, K velocity sweeps, filter,
collide).  Inputs are resident in HBM before timing starts.

Prints one JSON line: MLUPS of the FP32 step (the headline), the FP64 step,
the roofline of the dominant kernel (the fused collide) from HIP events on the
library's stream, the adjoint's cost against the forward step on the
closed-box rising bubble (256 x 1024), and the CPU oracle's rate on a bounded
sample.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# Algorithmic bytes of the collide pass per node, in values (8 B FP64, 4 B FP32):
# reads f, g (18), phi, p~, u~ (2), u~^n (2) and writes f, g (18).
COLLIDE_VALUES = 42
# Whole coupled step, pass model (values per node, each pass reading its inputs and
# writing its outputs once): gather 22 (18 populations in, phi_bar, p, j out); FD 8 over
# the three stages; velocity 8 per sweep; filter 6; collide 42 (94 at K = 2).  The
# two-sweep velocity kernel reads its inputs once, so the step moves 86 at K = 2.
def step_values(K):
    return 22 + 8 + 8 * K + 6 + 42


# Compulsory traffic of a coupled step if everything were fused: the state f*, g*
# and u~ read once and written once (20 + 20 values).
FLOOR_VALUES = 40


PROFILE_DIR = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILE_DIR, "k_collide_bubbles4096_hbm_traffic.md")
# what determines the collide kernel's code and launch shape: its source and
# helpers (tile shapes included) and the compiler flags
KERNEL_SOURCES = ["csrc/lbm2p_kernels.h", "csrc/lbm2p_math.h", "build.py"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1812_02459_amd", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per collide launch from the committed rocprofv3 counter summary,
    or None when the kernel sources changed after the counters were taken."""
    try:
        for line in open(TRAFFIC_FILE):
            if line.startswith("traffic_json: "):
                d = json.loads(line[len("traffic_json: "):])
                if d.get("source_sha256") == kernel_source_hash():
                    return d["bytes_per_launch"]
    except OSError:
        pass
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096, help="lattice side")
    ap.add_argument("--bubbles", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-side", type=int, default=1024, help="CPU sample window side")
    ap.add_argument("--cpu-steps", type=int, default=120)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the compact-filter and CH-only throughput legs")
    ap.add_argument("--adj-steps", type=int, default=640, help="steps of the adjoint timing")
    ap.add_argument("--variants-only", action="store_true",
                    help="only the compact-filter and CH-only legs (prints their JSON object)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint cost (prints its JSON object), e.g. for a kernel trace")
    return ap.parse_args()


def run_precision(wl, precision, steps, warmup, params=None):
    """Time `steps` steps after `warmup` untimed ones, then the average launch time
    of each pass of the step (10 more steps per pass, outside the timed region)."""
    import torch
    from paper_1812_02459_amd.binding import Sim
    params = params or wl.params
    sim = Sim(params, precision=precision)
    sim.init(wl.phi0, wl.ux0, wl.uy0, wl.p0)
    torch.cuda.synchronize()
    sim.step(warmup)
    torch.cuda.synchronize()
    diag0 = sim.volume()
    sim.profile("collide")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    coll_ms, coll_n = sim.profile_read()
    sim.profile(None)
    diag = sim.volume()
    passes = {}
    for name in ("gather", "fd", "vel", "filter", "collide"):
        sim.profile(name)
        sim.step(10)
        torch.cuda.synchronize()
        ms, n = sim.profile_read()
        if n:
            passes[name] = round(ms / n, 4)
    sim.profile(None)
    nodes = params["nx"] * params["ny"]
    dt = (t1 - t0) / steps
    esz = 4 if precision else 8
    avg_coll = coll_ms / max(coll_n, 1) * 1e-3
    coll_bytes = COLLIDE_VALUES * esz * nodes
    res = dict(
        mlups=nodes / dt / 1e6,
        ms_per_step=dt * 1e3,
        collide_ms=avg_coll * 1e3,
        collide_launches=coll_n,
        collide_gbps=coll_bytes / avg_coll / 1e9,
        collide_bytes=coll_bytes,
        step_gbps_model=step_values(params["K"]) * esz * nodes / dt / 1e9,
        step_gbps_floor=FLOOR_VALUES * esz * nodes / dt / 1e9,
        pass_ms=passes,
        finite=bool(diag["finite"]),
        sum_phi_drift=diag["sum_phi"] - diag0["sum_phi"],
        max_u=diag["max_u"],
        phi_range=[diag["min_phi"], diag["max_phi"]],
    )
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return res


def variant_legs(wl, steps, warmup, fp64=True):
    """The step's other configurations, not the headline: the compact-filter
    variant on the same bubble workload, and the CH-only step (prescribed
    single-vortex velocity, no velocity or filter passes) on the same lattice
    and on 128^2."""
    from paper_1812_02459_amd import inputs as I
    keep = ("mlups", "ms_per_step", "pass_ms", "finite")
    precs = (1, 0) if fp64 else (1,)
    out = {}
    pc = dict(wl.params)
    pc["compact"] = True
    out["compact_filter"] = {
        "workload": "same bubble ensemble, compact tridiagonal filter "
                    f"(N={pc['compact_n']}, alpha={pc['compact_alpha']}) in place of SF-11",
        **{("fp32" if pr else "fp64"): {k: v for k, v in run_precision(wl, pr, steps, warmup, pc).items()
                                        if k in keep} for pr in precs}}
    for n in (wl.params["nx"], 128):
        v = I.vortex(n=n)
        out[f"ch_only_{n}"] = {
            "workload": f"single vortex {n}x{n}, CH-only (prescribed velocity)",
            **{("fp32" if pr else "fp64"): {k: val for k, val in run_precision(v, pr, steps, warmup).items()
                                            if k in keep} for pr in precs}}
    return out


def adjoint_cost(precision, nsteps, k=64, warmup=64, compact=False):
    """Forward step time against the adjoint's time per step (segment recompute
    plus reverse sweep, checkpoints every k steps) on the closed-box rising
    bubble, 256 x 1024, R = 32, loss seed 2 (phi_T - phi*)/N; with compact,
    the compact tridiagonal filter (N = 5, alpha = 0.45) in place of SF-11."""
    import torch
    from paper_1812_02459_amd import inputs as I
    from paper_1812_02459_amd.binding import Sim
    wl = I.rising_bubble()
    if compact:
        wl.params = dict(wl.params, compact=True, compact_n=5, compact_alpha=0.45)
    sim = Sim(wl.params, precision=precision)
    sim.init(wl.phi0, wl.ux0, wl.uy0, wl.p0)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(nsteps)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / nsteps
    sim.close()
    sim = Sim(wl.params, precision=precision)
    sim.init(wl.phi0, wl.ux0, wl.uy0, wl.p0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.record(nsteps, k)
    torch.cuda.synchronize()
    t_rec = (time.perf_counter() - t0) / nsteps
    phiT = sim.moments()["phi"]
    seed = 2.0 * (phiT - torch.tanh(phiT)) / phiT.numel()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = sim.adjoint(dL_dphi=seed, want_phi0=True)
    torch.cuda.synchronize()
    t_adj = (time.perf_counter() - t0) / nsteps
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return dict(fwd_us_per_step=round(t_fwd * 1e6, 2), record_us_per_step=round(t_rec * 1e6, 2),
                adj_us_per_step=round(t_adj * 1e6, 2), ratio=round(t_adj / t_fwd, 3),
                steps=nsteps, ckpt_every=k, finite=bool(np.isfinite(g["sigma"])))


def copy_bandwidth():
    """Device copy rates (GB/s, read + write) of 1 GiB: the library's streaming
    copy (16-byte nontemporal accesses, the ceiling the kernels are measured
    against) and torch's copy_ (context)."""
    import torch
    from paper_1812_02459_amd import binding as B
    n = 1 << 28  # 1 GiB of float32
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream().cuda_stream
    kinds = {
        "stream": lambda: B.lbm2p_stream_copy(a.data_ptr(), b.data_ptr(), 4 * n, stream),
        "torch": lambda: b.copy_(a),
    }
    out = {}
    for name, fn in kinds.items():
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        out[name] = 2 * n * 4 / ((time.perf_counter() - t0) / reps) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def cpu_baseline(wl, side, steps):
    """The oracle, untuned, on a side x side window of the same initial field and
    parameters (periodic window), timed on this host's cores."""
    import torch
    import oracle
    # the host's CPU share (OMP_NUM_THREADS where the job sets it), else every core
    torch.set_num_threads(int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1))
    p = dict(wl.params)
    p["nx"] = p["ny"] = side
    prm = oracle.Params(**p)
    t = lambda a: torch.tensor(a[:side, :side].copy(), dtype=torch.float64)
    st = oracle.init_state(t(wl.phi0), t(wl.ux0), t(wl.uy0), t(wl.p0), prm)
    st = oracle.step_once(st, prm)                      # warm-up
    t0 = time.perf_counter()
    for _ in range(steps):
        st = oracle.step_once(st, prm)
    dt = time.perf_counter() - t0
    # the model name (some hosts report only "AMD EPYC") with family / model /
    # stepping, which name the core generation where the name does not
    cpu = ""
    try:
        info = {}
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                info.setdefault(k.strip(), v.strip())
        cpu = "%s (family %s, model %s, stepping %s; %d logical CPUs)" % (
            info.get("model name", "?"), info.get("cpu family", "?"), info.get("model", "?"),
            info.get("stepping", "?"), os.cpu_count() or 0)
    except OSError:
        pass
    return dict(value=side * side * steps / dt / 1e6, unit="MLUPS",
                cores=torch.get_num_threads(), cpu=cpu, kind="oracle",
                sample=f"{side}x{side} window of the 4096^2 bubble field, same parameters, "
                       f"FP64, {steps} timed steps after 1 warm-up step ({dt:.1f} s)")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU slab decomposition is designed but not implemented.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1812_02459_amd import inputs as I
    if args.adjoint_only:
        res = {"fp32": adjoint_cost(1, args.adj_steps)}
        if not args.no_fp64:
            res["fp64"] = adjoint_cost(0, args.adj_steps)
        res["fp32_compact_filter"] = adjoint_cost(1, args.adj_steps, compact=True)
        res["fp32_all_steps_kept"] = adjoint_cost(1, args.adj_steps, k=args.adj_steps)
        if not args.no_fp64:
            res["fp64_all_steps_kept"] = adjoint_cost(0, args.adj_steps, k=args.adj_steps)
        print(json.dumps({"adjoint": res}), flush=True)
        return
    t0 = time.perf_counter()
    wl = I.bubble_ensemble(n=args.n, nb=args.bubbles, seed=0, steps=args.steps)
    print(f"# workload built in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if args.variants_only:
        print(json.dumps({"variants": variant_legs(wl, args.steps, args.warmup,
                                                   not args.no_fp64)}), flush=True)
        return
    r32 = run_precision(wl, 1, args.steps, args.warmup)
    print(f"# fp32: {r32['mlups']:.0f} MLUPS, collide {r32['collide_ms']:.3f} ms "
          f"({r32['collide_gbps']:.0f} GB/s)", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = run_precision(wl, 0, args.steps, args.warmup)
        print(f"# fp64: {r64['mlups']:.0f} MLUPS, collide {r64['collide_ms']:.3f} ms "
              f"({r64['collide_gbps']:.0f} GB/s)", file=sys.stderr, flush=True)
    adj = None
    if not args.no_adjoint:
        adj = {"workload": "closed-box rising bubble 256x1024, R=32, walls on all sides, "
                           "rho1/rho2=1000, Eo=10, Re=35, U_g=2e-3; adjoint time = segment "
                           "recompute + reverse sweep, per step",
               "fp32": adjoint_cost(1, args.adj_steps)}
        if not args.no_fp64:
            adj["fp64"] = adjoint_cost(0, args.adj_steps)
        adj["fp32_compact_filter"] = adjoint_cost(1, args.adj_steps, compact=True)
        # every step's intermediates kept (checkpoint interval = run length: one
        # segment, kept by the record, so the adjoint recomputes nothing);
        # workspace 8.2 GB FP32, 16.4 GB FP64 for 640 steps at 256 x 1024
        adj["fp32_all_steps_kept"] = adjoint_cost(1, args.adj_steps, k=args.adj_steps)
        if not args.no_fp64:
            adj["fp64_all_steps_kept"] = adjoint_cost(0, args.adj_steps, k=args.adj_steps)
        print(f"# adjoint/forward: fp32 {adj['fp32']['ratio']:.2f}"
              + (f", fp64 {adj['fp64']['ratio']:.2f}" if "fp64" in adj else "")
              + f", fp32 compact filter {adj['fp32_compact_filter']['ratio']:.2f}"
              + f"; all steps kept: fp32 {adj['fp32_all_steps_kept']['ratio']:.2f}"
              + (f", fp64 {adj['fp64_all_steps_kept']['ratio']:.2f}"
                 if "fp64_all_steps_kept" in adj else ""),
              file=sys.stderr, flush=True)
    variants = None
    if not args.no_variants:
        variants = variant_legs(wl, min(args.steps, 300), min(args.warmup, 20), not args.no_fp64)
        print("# variants: " + ", ".join(
            f"{k} fp32 {v['fp32']['mlups']:.0f} MLUPS" for k, v in variants.items()),
            file=sys.stderr, flush=True)
    copies = copy_bandwidth()
    copy_gbps = copies["stream"]
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_side, args.cpu_steps)
        print(f"# cpu oracle: {cpu['value']:.3f} MLUPS on {cpu['cores']} threads",
              file=sys.stderr, flush=True)
    nodes = args.n * args.n
    traffic = measured_traffic() if args.n == 4096 else None
    out = {
        "metric": "coupled-step MLUPS + %HBM roofline, FP32 vs FP64 at stated error; "
                  "adjoint/forward time",
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"bubble ensemble {args.n}x{args.n} periodic, {args.bubbles} gas "
                        "bubbles R in [10,60], rho1/rho2=1000, mu1/mu2=100, Eo=10, Re=35, "
                        "W=4, M=0.02, lambda=0.005, SF-11 a=0.5, K=2",
            "nodes": nodes,
            "precision_headline": "fp32",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_collide (fused MRT collide + in-place stream of f and g)",
            "achieved": round(r32["collide_gbps"], 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(r32["collide_gbps"] / HBM_PEAK_GBPS, 4),
            "traffic": (round(traffic / (r32["collide_ms"] * 1e-3) / 1e9, 1)
                        if traffic else None),
            "traffic_bytes_per_launch": traffic,
            "bytes_per_launch": r32["collide_bytes"],
            "avg_launch_ms": round(r32["collide_ms"], 4),
            "frac_of_device_copy": round(r32["collide_gbps"] / copy_gbps, 4),
        },
        "step": {
            "fp32": {k: r32[k] for k in ("mlups", "ms_per_step", "step_gbps_model", "pass_ms",
                                          "finite", "sum_phi_drift", "max_u", "phi_range")},
        },
        "adjoint": adj,
        "variants": variants,
        "copy_GBps": round(copy_gbps, 1),
        "torch_copy_GBps": round(copies["torch"], 1),
        "cpu_baseline": cpu,
    }
    if r64 is not None:
        out["step"]["fp64"] = {k: r64[k] for k in ("mlups", "ms_per_step", "step_gbps_model",
                                                    "pass_ms", "finite", "sum_phi_drift", "max_u",
                                                    "phi_range", "collide_ms", "collide_gbps")}
        out["step"]["fp64"]["collide_frac"] = round(r64["collide_gbps"] / HBM_PEAK_GBPS, 4)
    # the whole step against the roofline: the pass model (94 values per node at
    # K = 2) and the compulsory floor (40), each against the 8 TB/s peak and the
    # measured device-copy bandwidth
    for name, r in (("fp32", r32), ("fp64", r64)):
        if r is None:
            continue
        out["step"][name].update(
            step_gbps_floor=r["step_gbps_floor"],
            pct_peak_pass_model=round(100 * r["step_gbps_model"] / HBM_PEAK_GBPS, 1),
            pct_peak_floor=round(100 * r["step_gbps_floor"] / HBM_PEAK_GBPS, 1),
            pct_copy_pass_model=round(100 * r["step_gbps_model"] / copy_gbps, 1),
            pct_copy_floor=round(100 * r["step_gbps_floor"] / copy_gbps, 1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
