"""Throughput benchmark of the Method-B convergence path on one MI355X.

Workload (the light-cone configuration): a uniform periodic 512^3 grid of
1 Gpc/h holding an FP32 potential from a seeded lognormal density, 2048^2
rays over 5 x 5 deg from the box corner to chi_s = chi(z = 1), advanced in
20 chi segments (one per synthetic N-body step, potential rescaled by the
linear growth of each step).  One step = the whole light cone: for each of the
20 segments, build the vertex tensor of that step's potential and march every
ray through the segment.  The FP32-Kahan path is timed and compared with the
plain FP64 path on the same inputs; the FP64 CPU oracle is timed on a bounded
sample of the same workload on the host cores.

Prints one JSON line (rank 0).
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
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_CROSSING = {"fp32": 96, "fp64": 192}    # 4 new corners x 6 components
BYTES_PER_VERTEX = {"fp32": 4 + 24, "fp64": 4 + 48}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--rays", type=int, default=2048)
    ap.add_argument("--segments", type=int, default=20)
    ap.add_argument("--persistent", type=int, default=-1)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=8192)
    ap.add_argument("--profile-steps", action="store_true",
                    help="short run for profilers: skip the CPU baseline and the FP64 leg")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB device-to-device (a plain "
                         "copy kernel that calibrates the profiler's byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.profile_steps:
        args.no_fp64 = True
        args.no_cpu = True

    import torch
    from paper_1601_02012_amd import api, inputs as I

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, box = args.n, 1000.0
    nray = args.rays
    fov = math.radians(5.0)
    log(f"generating inputs: {n}^3 lognormal potential, {nray}^2 rays, {args.segments} segments")
    t0 = time.time()
    phi0 = I.config2_phi0(n, box)
    segs = I.lightcone_segments(args.segments)
    chi_s = I.chi_of_z(1.0)
    dirs = I.fov_directions((0.0, 0.0, 1.0), fov, fov, nray, nray)
    log(f"inputs ready in {time.time() - t0:.1f}s")

    phi0_d = torch.as_tensor(phi0, device=dev)
    phis = [(phi0_d * s).to(torch.float32).contiguous() for (_, _, s) in segs]
    del phi0_d
    dirs_d = torch.as_tensor(dirs, device=dev)
    grids = [api.Grid(p, box) for p in phis]
    plan = api.Plan()
    bundles = [[api.RayBundle(dirs_d, nray, nray, chi_s, hi, lo)] for (hi, lo, _) in segs]
    obs = (0.0, 0.0, 0.0)
    nr = nray * nray
    stream = torch.cuda.current_stream()

    def run_step(tensor, kap, comp, st, events=None):
        for k in range(len(segs)):
            if events is not None:
                events[k][0].record(stream)
            tensor.build(grids[k])
            if events is not None:
                events[k][1].record(stream)
            api.trace(plan, tensor, bundles[k], obs, kappa=kap, kappa_comp=comp, status=st,
                      persistent=args.persistent)
            if events is not None:
                events[k][2].record(stream)

    results = {}
    for prec in (["fp32"] + ([] if args.no_fp64 else ["fp64"])):
        t = api.TidalTensor(grids[0], prec)
        fp32 = prec == "fp32"
        kdt = torch.float32 if fp32 else torch.float64
        kap = torch.zeros(nr, dtype=kdt, device=dev)
        comp = torch.zeros(nr, dtype=torch.float32, device=dev) if fp32 else None
        st = torch.zeros(nr, dtype=torch.int32, device=dev)
        # crossing count of one light cone (untimed debug pass)
        total_cross = 0
        for k in range(len(segs)):
            t.build(grids[k])
            o = api.trace(plan, t, bundles[k], obs, debug=True, persistent=0)
            total_cross += int(o.count.sum().item())
        log(f"{prec}: {total_cross:.4e} crossings per light cone")
        for w in range(args.warmup):
            kap.zero_()
            if comp is not None:
                comp.zero_()
            run_step(t, kap, comp, st)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in segs]
        step_ms, build_ms, march_ms = [], [], []
        for s in range(args.steps):
            kap.zero_()
            if comp is not None:
                comp.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run_step(t, kap, comp, st, ev)
            torch.cuda.synchronize()
            step_ms.append((time.perf_counter() - t0) * 1e3)
            build_ms.append(sum(e[0].elapsed_time(e[1]) for e in ev))
            march_ms.append(sum(e[1].elapsed_time(e[2]) for e in ev))
            log(f"{prec} step {s}: {step_ms[-1]:.2f} ms (build {build_ms[-1]:.2f}, "
                f"march {march_ms[-1]:.2f})")
        stat = st.cpu().numpy()
        results[prec] = dict(cross=total_cross, step_ms=float(np.mean(step_ms)),
                             build_ms=float(np.mean(build_ms)), march_ms=float(np.mean(march_ms)),
                             kappa=kap.double().cpu().numpy(), status_ok=bool(np.all(stat == 0)))
        t.close()
        del kap, comp, st
        torch.cuda.empty_cache()

    if args.copy_probe_mib:
        nb = args.copy_probe_mib * (1 << 20)
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB x 3")
        del src, dst

    r32 = results["fp32"]
    value = r32["cross"] / (r32["step_ms"] * 1e-3)
    nseg = len(segs)
    march_launch_ms = r32["march_ms"] / nseg
    cross_per_launch = r32["cross"] / nseg
    achieved = BYTES_PER_CROSSING["fp32"] * cross_per_launch / (march_launch_ms * 1e-3) / 1e9
    out = {
        "metric": "ray-cell crossings/sec and HBM GB/s, FP32-comp vs FP64 at 1e-5 rel kappa err",
        "value": value,
        "unit": "crossings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"uniform periodic {n}^3 grid, box 1000 Mpc/h, FP32 lognormal "
                               f"potential, {nray}x{nray} rays over 5x5 deg, {nseg} chi segments "
                               "to z=1 (tensor rebuilt per segment), FP32-Kahan march",
                   "grid": n, "rays": nr, "segments": nseg, "chi_s": chi_s},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "march_uniform (FP32-Kahan)",
                     "bytes_per_crossing": BYTES_PER_CROSSING["fp32"],
                     "launch_ms": march_launch_ms, "crossings_per_launch": cross_per_launch},
        "march_crossings_per_s": r32["cross"] / (r32["march_ms"] * 1e-3),
        "tensor_build_ms_per_segment": r32["build_ms"] / nseg,
        "tensor_build_gbs": BYTES_PER_VERTEX["fp32"] * n ** 3 / (r32["build_ms"] / nseg * 1e-3) / 1e9,
        "all_rays_ok": r32["status_ok"],
    }
    if "fp64" in results:
        r64 = results["fp64"]
        out["fp64_crossings_per_s"] = r64["cross"] / (r64["step_ms"] * 1e-3)
        out["speedup_vs_fp64"] = r64["step_ms"] / r32["step_ms"]
        out["fp64_march_crossings_per_s"] = r64["cross"] / (r64["march_ms"] * 1e-3)
        out["crossings_equal_fp32_fp64"] = r64["cross"] == r32["cross"]
        ref = r64["kappa"]
        err = np.abs(r32["kappa"] - ref)
        lim = np.maximum(1e-5 * np.abs(ref), 1e-7)
        out["kappa_fp32_vs_fp64"] = {"max_err_over_tol": float(np.max(err / lim)),
                                     "max_abs_err": float(err.max()),
                                     "rms_kappa": float(np.sqrt(np.mean(ref ** 2)))}
    if not args.no_cpu:
        out["cpu_baseline"], out["oracle_parity_sample"] = cpu_baseline(
            phis, segs, dirs, chi_s, box, obs, args.cpu_rays, results)
    print(json.dumps(out), flush=True)


def cpu_baseline(phis, segs, dirs, chi_s, box, obs, n_sample, results):
    """FP64 oracle on the host: the vertex tensor of the last segment's
    potential, then a deterministic sample of rays through that segment."""
    import torch
    from oracle import oracle as O
    k = len(segs) - 1
    hi, lo, _ = segs[k]
    phi = phis[k].double().cpu().numpy()
    n = phi.shape[0]
    cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    tv = O.vertex_tensor(phi)
    t_tensor = time.perf_counter() - t0
    rng = np.random.default_rng(12345)
    perm = rng.permutation(dirs.shape[0])
    # pilot run, then size the sample to about 15 s of oracle work
    pilot = np.sort(perm[:min(n_sample, dirs.shape[0])])
    t0 = time.perf_counter()
    rp = O.trace_uniform(n, box, obs, dirs[pilot], chi_s, hi, lo, tv=tv, threads=cores)
    tp = max(time.perf_counter() - t0, 1e-3)
    want = int(len(pilot) * min(15.0 / tp, 1e6))
    sel = np.sort(perm[:max(len(pilot), min(want, dirs.shape[0]))])
    t0 = time.perf_counter()
    r = O.trace_uniform(n, box, obs, dirs[sel], chi_s, hi, lo, tv=tv, threads=cores)
    t_trace = time.perf_counter() - t0
    cross = int(r.ncross.sum())
    del rp
    log(f"oracle: tensor {t_tensor:.1f}s, {len(sel)} rays / {cross} crossings in {t_trace:.1f}s")
    # GPU FP32 segment result for the same rays and segment (parity sample)
    from paper_1601_02012_amd import api
    g = api.Grid(phis[k], box)
    t = api.TidalTensor(g, "fp32").build()
    plan = api.Plan()
    b = api.RayBundle(torch.as_tensor(dirs[sel]).cuda(), len(sel), 1, chi_s, hi, lo)
    o = api.trace(plan, t, [b], obs, debug=True)
    gk = o.kappa.double().cpu().numpy()
    same = bool(np.array_equal(o.hash.cpu().numpy().view(np.uint64), r.hash))
    err = np.abs(gk - r.kappa)
    lim = np.maximum(1e-5 * np.abs(r.kappa), 1e-7)
    t.close()
    cb = {"value": cross / t_trace, "unit": "crossings/s", "cores": cores, "kind": "oracle",
          "sample": f"{len(sel)} rays of the last chi segment ({cross} crossings), FP64 C oracle "
                    f"with OpenMP; its {n}^3 vertex tensor took {t_tensor:.1f}s (not included)",
          "tensor_build_s": t_tensor}
    par = {"rays": len(sel), "crossing_hashes_equal": same,
           "max_err_over_tol": float(np.max(err / lim))}
    return cb, par


if __name__ == "__main__":
    main()
