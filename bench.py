"""Throughput benchmark of the Method-B convergence path on one MI355X.

Headline workload (the light cone): a uniform periodic 512^3 grid of 1 Gpc/h
holding an FP32 potential from a seeded lognormal density, 2048^2 rays over
5 x 5 deg from the box corner to chi_s = chi(z = 1), advanced in 20 chi
segments (one per synthetic N-body step, potential rescaled by the linear
growth of each step).  One step = the whole light cone: for each segment,
build the vertex tensor of that step's potential over the whole grid and march
every ray through the segment.  The FP32-Kahan path is timed against the plain
FP64 path on the same inputs.

Further legs (reported beside the headline, not in ``value``): the AMR octree
(256^3 base + 4 levels, 4096^2 rays to z = 1) and the batched set of 64
uneven bundles through it in one persistent launch replayed from a HIP graph.
The FP64 CPU oracle is timed on a bounded sample of the light cone.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_CROSSING = {"fp32": 96, "fp64": 192}     # 4 new corners x 6 components
# MI355X vector peak: 256 CUs x 4 SIMDs x 32 FP32 lanes x 2 (FMA) x 2.4 GHz;
# FP64 runs at half that rate
PEAK_FP32_TFLOPS = 157.3
# arithmetic of one single-face crossing of the FP32-Kahan march, counted from
# the method (an FMA counts two): the three-point Gauss integral of the cell
# (102, scale included), four corner projections P:T (4 x 11), the Kahan
# update (4) and the local exit coordinates (6) in FP32; the exit selection
# and tie tests (6 comparisons), exit coordinates (3), the piece length and
# chi_s - chi_B (2) and the next plane's parameter (2) in FP64
FLOPS_PER_CROSSING = {"fp32": 156, "fp64": 13}
# arithmetic of one crossing of the adjoint scatter, counted the same way: per
# Gauss node the node's chi and kernel weight (6), its local coordinates (6),
# the eight trilinear corner weights scaled by the node weight (3 + 2 + 4 + 8)
# and their accumulation (8), after the piece's three coordinate differences
# (3); when a face retires, its four corners' weights times the six projection
# factors and their sums (24 + 24); the walk's 13 FP64 operations as above
ADJ_FLOPS_PER_CROSSING = {"fp32": 3 * (6 + 6 + 17 + 8) + 3 + 48, "fp64": 13}
BYTES_PER_VERTEX = {"fp32": 4 + 24, "fp64": 4 + 48}  # potential in, 6 components out
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "march_uniform_lightcone_traffic.md")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "march_uniform_lightcone_counters.md")
WAVE_FILE = os.path.join(ROOT, "profiles", "wave_state_counters.md")
MARCH_SOURCES = ["paper_1601_02012_amd/csrc/rr_march_uniform.hip",
                 "paper_1601_02012_amd/csrc/rr_ray.hpp",
                 "paper_1601_02012_amd/csrc/rr_internal.hpp"]
ADJOINT_FILE = os.path.join(ROOT, "profiles", "adjoint_scatter_counters.md")
ADJOINT_SOURCES = ["paper_1601_02012_amd/csrc/rr_adjoint_uniform.hip",
                   "paper_1601_02012_amd/csrc/rr_ray.hpp",
                   "paper_1601_02012_amd/csrc/rr_internal.hpp"]


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def source_hash(files=MARCH_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def march_source_hash():
    return source_hash(MARCH_SOURCES)


def profile_figures(paths=(TRAFFIC_FILE, COUNTERS_FILE, WAVE_FILE), files=MARCH_SOURCES,
                    tag="march_source_sha256_16"):
    """Figures from the committed rocprofv3 summaries (for the march: HBM bytes per
    launch, L2 hit fraction, VALU busy fraction, VALU instructions per crossing), each
    kept only if the summary was taken on the current source of that kernel."""
    src = source_hash(files)
    out = {}
    for path in paths:
        if not os.path.exists(path):
            continue
        txt = open(path).read()
        m_src = re.search(tag + r":\s*([0-9a-f]+)", txt)
        if not m_src or m_src.group(1) != src:
            continue
        for key, val in re.findall(r"^(\w+):\s*([0-9.eE+-]+)\s*$", txt, re.M):
            out[key] = float(val)
    return out


def timed(fn, steps, warmup, label):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ms = []
    for s in range(steps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
        log(f"{label} step {s}: {ms[-1]:.2f} ms")
    return float(np.mean(ms))


def lightcone_leg(args, api, I, torch, dev):
    n, box = args.n, 1000.0
    nray = args.rays
    fov = math.radians(5.0)
    log(f"light cone: {n}^3 lognormal potential, {nray}^2 rays, {args.segments} segments")
    delta0, phi0 = I.config2_fields(n, box)
    segs = I.lightcone_segments(args.segments)
    chi_s = I.chi_of_z(1.0)
    dirs = I.fov_directions((0.0, 0.0, 1.0), fov, fov, nray, nray)
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
    results = {}
    for prec in (["fp32"] + ([] if args.no_fp64 else ["fp64"])):
        t = api.TidalTensor(grids[0], prec)
        fp32 = prec == "fp32"
        kap = torch.zeros(nr, dtype=torch.float32 if fp32 else torch.float64, device=dev)
        comp = torch.zeros(nr, dtype=torch.float32, device=dev) if fp32 else None
        st = torch.zeros(nr, dtype=torch.int32, device=dev)
        total_cross = 0
        shapes = []
        seg_hash = []
        for k in range(len(segs)):
            t.build(grids[k])
            o = api.trace(plan, t, bundles[k], obs, debug=True, persistent=0)
            total_cross += int(o.count.sum().item())
            if fp32:
                seg_hash.append((o.hash, o.count))   # kept on the device for the oracle check
            del o
            if args.tune_lightcone:
                shapes.append(plan.autotune(t, bundles[k], obs))
        log(f"{prec}: {total_cross:.4e} crossings per light cone; tuned shapes "
            f"{sorted(set((s['persistent'], s['block'], s['waves_per_cu']) for s in shapes))}")
        if prec == "fp32":
            # vertex box of every segment (geometry only: computed once, like the tables)
            boxes = [plan.vertex_box(t, bundles[k], obs) for k in range(len(segs))]
            frac = sum(int(np.prod(b[1])) for b in boxes) / (len(segs) * float(n) ** 3)
            log(f"vertex boxes cover {100 * frac:.2f}% of the grid over the light cone")
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in segs]
        for mode in ("whole", "box"):
            def step():
                kap.zero_()
                if comp is not None:
                    comp.zero_()
                for k in range(len(segs)):
                    ev[k][0].record(stream)
                    if mode == "whole":
                        t.build(grids[k])
                    else:
                        t.build_box(boxes[k][0], boxes[k][1], grid=grids[k])
                    ev[k][1].record(stream)
                    api.trace(plan, t, bundles[k], obs, kappa=kap, kappa_comp=comp, status=st,
                              persistent=-1 if args.tune_lightcone else 0)
                    ev[k][2].record(stream)

            step_ms = timed(step, args.steps, args.warmup, f"light cone {prec} {mode}")
            build_ms = sum(e[0].elapsed_time(e[1]) for e in ev)
            march_ms = sum(e[1].elapsed_time(e[2]) for e in ev)
            results[prec if mode == "whole" else prec + "_box"] = dict(
                cross=total_cross, step_ms=step_ms, build_ms=build_ms, march_ms=march_ms,
                kappa=kap.double().cpu().numpy(), status_ok=bool((st == 0).all().item()),
                shapes=[(s["persistent"], s["block"], s["waves_per_cu"]) for s in shapes],
                box_frac=frac, seg_hash=seg_hash)
        t.close()
        del kap, comp, st
        torch.cuda.empty_cache()
    if not args.no_method_a:
        results["method_a"] = method_a_leg(args, api, I, torch, dev, delta0, grids, segs,
                                           bundles, obs, results)
    if not args.no_sources:
        results["sources"] = sources_leg(args, api, I, torch, dev, grids, segs, bundles, obs,
                                         results)
    if not args.no_isw:
        results["isw"] = isw_leg(args, api, I, torch, dev, grids, segs, bundles, obs)
    if not args.no_adjoint:
        results["adjoint"] = adjoint_leg(args, api, I, torch, dev)
    del delta0
    if args.copy_probe_mib:
        nb = args.copy_probe_mib * (1 << 20)
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB x 3")
        del src, dst
    ctx = dict(phis=phis, segs=segs, dirs=dirs, chi_s=chi_s, box=box, obs=obs, n=n)
    return results, ctx


def method_a_leg(args, api, I, torch, dev, delta0, grids, segs, bundles, obs, results):
    """The same light cone with Method A (Eq. kappa2): per segment the vertex
    fields (c delta, grad Phi) and the march with the density and gradient
    kernels plus the segment's surface term; compared with Method B's map."""
    box = grids[0].box
    nr = bundles[0][0].n_rays
    dd = torch.as_tensor(delta0.astype(np.float32), device=dev)
    gd = api.Grid(dd, box, field="delta")
    t = api.TidalTensor(gd, "fp32")
    kap = torch.zeros(nr, dtype=torch.float32, device=dev)
    comp = torch.zeros(nr, dtype=torch.float32, device=dev)
    st = torch.zeros(nr, dtype=torch.int32, device=dev)
    c0 = I.poisson_coefficient()
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in segs]

    def step():
        kap.zero_()
        comp.zero_()
        for k, (_, _, sk) in enumerate(segs):
            ev[k][0].record(stream)
            t.build_method_a(gd, grids[k], c0 * sk)
            ev[k][1].record(stream)
            api.trace(api_plan[0], t, bundles[k], obs, kappa=kap, kappa_comp=comp, status=st,
                      persistent=0)
            ev[k][2].record(stream)

    api_plan = [api.Plan()]
    step_ms = timed(step, args.steps, args.warmup, "light cone fp32 Method A")
    build_ms = sum(e[0].elapsed_time(e[1]) for e in ev)
    march_ms = sum(e[1].elapsed_time(e[2]) for e in ev)
    ka = kap.double().cpu().numpy()
    kb = results["fp32"]["kappa"]
    t.close()
    del dd, kap, comp
    torch.cuda.empty_cache()
    cross = results["fp32"]["cross"]
    return {"workload": "the light cone with Method A (density and gradient terms, surface "
                        "term per segment), FP32-Kahan",
            "crossings_per_s": cross / (step_ms * 1e-3), "ms_per_step": step_ms,
            "fields_build_ms_per_segment": build_ms / len(segs),
            "march_crossings_per_s": cross / (march_ms * 1e-3),
            "all_rays_ok": bool((st == 0).all().item()),
            "kappa_vs_method_b": {
                "rms_diff_over_rms_kappa": float(np.sqrt(np.mean((ka - kb) ** 2))
                                                 / np.sqrt(np.mean(kb ** 2))),
                "correlation": float(np.corrcoef(ka, kb)[0, 1])}}


def isw_leg(args, api, I, torch, dev, grids, segs, bundles, obs):
    """The light cone with the ISW integrand (Sec. VII): per segment the vertex
    field of (Phi_k - Phi_k-1)/dt and the march with a constant kernel
    2 a_k / c, giving the ISW temperature shift of every ray."""
    steps = I.isw_steps(len(segs))
    box = grids[0].box
    nr = bundles[0][0].n_rays
    # the potential one step before the first segment
    prev0 = api.Grid((grids[0].values * float(steps[0][0] / steps[0][1])).contiguous(), box)
    gd = api.Grid(grids[0].values, box, field="phi_dot")
    t = api.TidalTensor(gd, "fp32")
    plan = api.Plan()
    out = torch.zeros(nr, dtype=torch.float32, device=dev)
    comp = torch.zeros(nr, dtype=torch.float32, device=dev)
    st = torch.zeros(nr, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in segs]
    cross = 0
    for k in range(len(segs)):
        t.build_isw(grids[k], grids[k - 1] if k else prev0, steps[k][2])
        cross += int(api.trace(plan, t, bundles[k], obs, quantity="scalar", debug=True,
                               persistent=0).count.sum().item())

    def step():
        out.zero_()
        comp.zero_()
        for k in range(len(segs)):
            ev[k][0].record(stream)
            t.build_isw(grids[k], grids[k - 1] if k else prev0, steps[k][2])
            ev[k][1].record(stream)
            api.trace(plan, t, bundles[k], obs, kappa=out, kappa_comp=comp, status=st,
                      quantity="scalar", kappa_scale=steps[k][3], persistent=0)
            ev[k][2].record(stream)

    ms = timed(step, args.steps, args.warmup, "light cone fp32 ISW")
    build_ms = sum(e[0].elapsed_time(e[1]) for e in ev)
    march_ms = sum(e[1].elapsed_time(e[2]) for e in ev)
    m = out.double().cpu().numpy()
    t.close()
    del out, comp, prev0
    torch.cuda.empty_cache()
    return {"workload": "the light cone with the ISW integrand: per segment the vertex field "
                        "of (Phi_k - Phi_k-1)/dt (growth-scaled potentials, dt from cosmic "
                        "time) and a constant kernel 2 a_k / c, FP32-Kahan",
            "crossings": cross, "ms_per_step": ms, "crossings_per_s": cross / (ms * 1e-3),
            "field_build_ms_per_segment": build_ms / len(segs),
            "march_crossings_per_s": cross / (march_ms * 1e-3),
            "all_rays_ok": bool((st == 0).all().item()),
            "map_mean": float(m.mean()), "map_rms": float(m.std())}


SOURCE_Z = [1.0, 0.9, 0.8, 0.7, 0.6, 0.5, 0.4, 0.3, 0.2, 0.1]


def sources_leg(args, api, I, torch, dev, grids, segs, bundles, obs, results):
    """The light cone for ten source redshifts (z = 1, 0.9, ..., 0.1): one walk
    that integrates int chi Q and int chi^2 Q and stops at every source
    (Eqs. Isources, Isources1), against one single-source trace per source."""
    nr = bundles[0][0].n_rays
    src = np.array([I.chi_of_z(z) for z in SOURCE_Z])
    t = api.TidalTensor(grids[0], "fp32")
    plan = api.Plan()
    st = None
    cross = 0
    for k in range(len(segs)):
        t.build(grids[k])
        st = api.trace_sources(plan, t, bundles[k], obs, src, state=st, debug=True, persistent=0)
        cross += int(st.count.sum().item())
    state = api.SourcesOutput(torch.zeros((nr, 4), dtype=torch.float32, device=dev),
                              torch.zeros((nr, len(src), 2), dtype=torch.float64, device=dev),
                              torch.zeros(nr, dtype=torch.int32, device=dev))
    kap = [None]

    def step():
        state.moments.zero_()
        state.pieces.zero_()
        for k in range(len(segs)):
            t.build(grids[k])
            api.trace_sources(plan, t, bundles[k], obs, src, state=state, persistent=0)
        kap[0] = api.kappa_from_pieces(plan, t, src, state)

    walk_ms = timed(step, args.steps, args.warmup, "light cone fp32, 10 sources in one walk")
    kw = kap[0].cpu().numpy()
    ok = bool((state.status == 0).all().item())
    # one trace per source: each source's rays from chi_s,j to the observer
    kaps = [torch.zeros(nr, dtype=torch.float32, device=dev) for _ in src]
    comps = [torch.zeros(nr, dtype=torch.float32, device=dev) for _ in src]
    per_bundles = []
    per_cross = 0
    for k, (hi, lo, _) in enumerate(segs):
        row = []
        for j, cs in enumerate(src):
            if cs > lo:
                b = bundles[k][0]
                row.append((j, [api.RayBundle(b.dirs, b.nx, b.ny, float(cs), min(hi, float(cs)),
                                              lo)]))
        per_bundles.append(row)
    for k in range(len(segs)):
        t.build(grids[k])
        for j, bb in per_bundles[k]:
            per_cross += int(api.trace(plan, t, bb, obs, debug=True, persistent=0)
                             .count.sum().item())

    def step_per_source():
        for j in range(len(src)):
            kaps[j].zero_()
            comps[j].zero_()
        for k in range(len(segs)):
            t.build(grids[k])
            for j, bb in per_bundles[k]:
                api.trace(plan, t, bb, obs, kappa=kaps[j], kappa_comp=comps[j], persistent=0)

    per_ms = timed(step_per_source, args.steps, args.warmup,
                   "light cone fp32, 10 sources one trace each")
    kp = torch.stack(kaps, 1).double().cpu().numpy()
    err = np.abs(kw - kp) / np.maximum(1e-5 * np.abs(kp), 1e-7)
    kb = results["fp32"]["kappa"]
    err0 = np.abs(kw[:, 0] - kb) / np.maximum(1e-5 * np.abs(kb), 1e-7)
    t.close()
    del state, kaps, comps
    torch.cuda.empty_cache()
    return {"workload": "the light cone with sources at z = 1.0, 0.9, ..., 0.1: one walk "
                        "integrating int chi Q and int chi^2 Q, stopping at each source, "
                        "tensor rebuilt over the whole grid every segment, FP32-Kahan",
            "sources_z": SOURCE_Z, "crossings": cross,
            "ms_per_step": walk_ms, "crossings_per_s": cross / (walk_ms * 1e-3),
            "per_source_ms_per_step": per_ms, "per_source_crossings": per_cross,
            "speedup_vs_one_trace_per_source": per_ms / walk_ms,
            "all_rays_ok": ok,
            "kappa_vs_one_trace_per_source_max_err_over_tol": float(err.max()),
            "kappa_z1_vs_headline_max_err_over_tol": float(err0.max()),
            "tolerance": "max(1e-5 |kappa|, 1e-7) per ray and source"}


def amr_leg(args, api, I, torch, dev):
    log("AMR octree: generating 256^3 base + 4 levels from 2^24 particles")
    t0 = time.time()
    case = I.config3()
    tr = case.tree
    log(f"AMR octree ready in {time.time() - t0:.1f}s: {tr.n_cells} cells, "
        f"levels {np.bincount(tr.cell_level).tolist()}")
    grid = api.Grid(torch.as_tensor(case.phi.astype(np.float32), device=dev), case.box,
                    n_base=tr.n, child_oct=torch.as_tensor(tr.child_oct, device=dev),
                    max_level=tr.max_level)
    tens = api.TidalTensor(grid, "fp32")
    plan = api.Plan()
    stream = torch.cuda.current_stream()
    out = {}
    # AMR light cone: 4096^2 rays over 10 x 10 deg to z = 1
    b = I.config3_rays(args.amr_rays)
    nr = b.nx * b.ny
    gb = [api.RayBundle(torch.as_tensor(b.dirs, device=dev), b.nx, b.ny, b.chi_s, b.chi_hi,
                        b.chi_lo)]
    tens.build(grid)
    cross = int(api.trace(plan, tens, gb, case.observer, debug=True, persistent=0)
                .count.sum().item())
    shape = None if args.no_tune else plan.autotune(tens, gb, case.observer)
    kap = torch.zeros(nr, dtype=torch.float32, device=dev)
    comp = torch.zeros(nr, dtype=torch.float32, device=dev)
    st = torch.zeros(nr, dtype=torch.int32, device=dev)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def step():
        kap.zero_()
        comp.zero_()
        e[0].record(stream)
        tens.build(grid)
        e[1].record(stream)
        api.trace(plan, tens, gb, case.observer, kappa=kap, kappa_comp=comp, status=st,
                  persistent=-1)
        e[2].record(stream)

    ms = timed(step, args.steps, args.warmup, "AMR")
    out["amr"] = {"workload": f"AMR octree 256^3 base + 4 levels ({tr.n_cells} cells), "
                              f"{b.nx}x{b.ny} rays over 10x10 deg to z=1, FP32-Kahan",
                  "crossings": cross, "ms_per_step": ms,
                  "crossings_per_s": cross / (ms * 1e-3),
                  "tensor_build_ms": e[0].elapsed_time(e[1]),
                  "march_ms": e[1].elapsed_time(e[2]),
                  "march_crossings_per_s": cross / (e[1].elapsed_time(e[2]) * 1e-3),
                  "all_rays_ok": bool((st == 0).all().item()), "tuned_shape": shape}
    del kap, comp, st, gb
    torch.cuda.empty_cache()
    # batched: 64 uneven bundles, one persistent launch, replayed from a graph
    specs = I.config4_specs()
    bundles, offset = [], 0
    for s in specs:
        bb = I.bundle_from_spec(s)
        bundles.append(api.RayBundle(torch.as_tensor(bb.dirs, device=dev), bb.nx, bb.ny,
                                     bb.chi_s, bb.chi_hi, bb.chi_lo, offset))
        offset += bb.nx * bb.ny
    nr = offset
    cross = int(api.trace(plan, tens, bundles, case.observer, debug=True, persistent=1)
                .count.sum().item())
    bshape = None if args.no_tune else plan.autotune(tens, bundles, case.observer)
    pers = -1 if bshape else 1
    kap = torch.zeros(nr, dtype=torch.float32, device=dev)
    comp = torch.zeros(nr, dtype=torch.float32, device=dev)
    st = torch.zeros(nr, dtype=torch.int32, device=dev)
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        api.trace(plan, tens, bundles, case.observer, kappa=kap, kappa_comp=comp, status=st,
                  persistent=pers)
        gs.synchronize()
        plan.graph_begin()
        api.trace(plan, tens, bundles, case.observer, kappa=kap, kappa_comp=comp, status=st,
                  persistent=pers)
        plan.graph_end()
    gs.synchronize()

    def bstep():
        kap.zero_()
        comp.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(gs):
            plan.graph_launch()
        gs.synchronize()

    ms = timed(bstep, args.steps, args.warmup, "batched")
    out["batched"] = {"workload": f"{len(specs)} bundles ({nr} rays, sides 256..2048, z_s "
                                  "0.5..2, FoV 1..10 deg, random centres) through the AMR "
                                  "octree, all bundles in each launch (autotuned shape and "
                                  "passes) replayed from a HIP graph, FP32-Kahan",
                      "tuned_shape": bshape,
                      "rays": nr, "crossings": cross, "ms_per_step": ms,
                      "crossings_per_s": cross / (ms * 1e-3),
                      "all_rays_ok": bool((st == 0).all().item())}
    tens.close()
    return out


def adjoint_leg(args, api, I, torch, dev):
    """The adjoint configuration: L = sum(w kappa) over a 1024^2 map through a
    256^3 FP32 potential; forward (tensor build + march) and backward
    (rr_trace_rays_adjoint: scatter of the corner weights, transpose of the
    vertex mean and stencil) timed per step, with the dot-product identity
    <A^T w, dPhi> = <w, A dPhi> checked on a random dPhi."""
    case, w = I.config5()
    b = case.bundles[0]
    n, box = case.n, case.box
    g = api.Grid(torch.as_tensor(case.phi, device=dev), box)
    t = api.TidalTensor(g, "fp32")
    plan = api.Plan()
    gb = [api.RayBundle(torch.as_tensor(b.dirs, device=dev), b.nx, b.ny, b.chi_s, b.chi_hi,
                        b.chi_lo)]
    wt = torch.as_tensor(w, dtype=torch.float32, device=dev)
    nr = b.nx * b.ny
    t.build(g)
    cross = int(api.trace(plan, t, gb, case.observer, debug=True, persistent=0)
                .count.sum().item())
    kap = torch.zeros(nr, dtype=torch.float32, device=dev)
    comp = torch.zeros(nr, dtype=torch.float32, device=dev)
    grad = torch.zeros((n, n, n), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def step():
        kap.zero_()
        comp.zero_()
        grad.zero_()
        ev[0].record(stream)
        t.build(g)
        api.trace(plan, t, gb, case.observer, kappa=kap, kappa_comp=comp, persistent=0)
        ev[1].record(stream)
        api.trace_adjoint(plan, t, g, gb, case.observer, wt, dl_dphi=grad)
        ev[2].record(stream)

    ms = timed(step, args.steps, args.warmup, "adjoint (forward + backward)")
    fwd_ms = ev[0].elapsed_time(ev[1])
    bwd_ms = ev[1].elapsed_time(ev[2])
    # dot-product identity on a random perturbation (kappa is linear in Phi)
    rng = np.random.default_rng(12345)
    dphi = torch.as_tensor(rng.standard_normal((n, n, n)).astype(np.float32) * 1e-5, device=dev)
    gd = api.Grid(dphi, box)
    kd = api.trace(plan, t.build(gd), gb, case.observer, persistent=0).kappa.double()
    lhs = float(torch.dot(wt.double(), kd).item())
    rhs = float(torch.dot(grad.double().flatten(), dphi.double().flatten()).item())
    t.close()
    del grad, kap, comp, dphi
    torch.cuda.empty_cache()
    flops_eq = ADJ_FLOPS_PER_CROSSING["fp32"] + 2 * ADJ_FLOPS_PER_CROSSING["fp64"]
    achieved = flops_eq * cross / (bwd_ms * 1e-3) / 1e12
    # the scatter's atomic bytes from the committed counter summary (same source only)
    prof = profile_figures((ADJOINT_FILE,), ADJOINT_SOURCES, "adjoint_source_sha256_16")
    lam = 6 * n ** 3 * 4   # dL/dLambda: six FP32 components per vertex
    return {"workload": "adjoint: L = sum(w kappa), w ~ N(0,1), 1024x1024 rays over 5x5 deg "
                        "to chi_s = 256 Mpc/h through a 256^3 FP32 Gaussian potential (box "
                        "256 Mpc/h); backward through the march, the vertex mean and the "
                        "stencil to dL/dPhi",
            "crossings": cross, "ms_per_step": ms, "forward_ms": fwd_ms, "backward_ms": bwd_ms,
            "backward_crossings_per_s": cross / (bwd_ms * 1e-3),
            "dot_product_identity_rel_diff": abs(lhs - rhs) / max(abs(lhs), abs(rhs), 1e-300),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                         "flops_per_crossing": {**ADJ_FLOPS_PER_CROSSING,
                                                "fp32_equivalent": flops_eq},
                         "kernel": "the backward call (scatter_kernel, then transpose_kernel), "
                                   "timed with HIP events on its stream",
                         "scatter_atomic_bytes_per_launch": prof.get(
                             "scatter_write_bytes_per_launch"),
                         "lambda_bytes": lam,
                         "scatter_atomic_bytes_over_lambda": (
                             prof["scatter_write_bytes_per_launch"] / lam
                             if "scatter_write_bytes_per_launch" in prof else None),
                         "scatter_valu_insts_per_wave_crossing": prof.get(
                             "scatter_valu_insts_per_wave_crossing")}}


def amr_profile(args, api, I, torch, dev):
    """The AMR map alone, for profilers: one tensor build and two timed marches
    of all 4096^2 rays with a fixed launch shape (one-wavefront-per-tile,
    256-thread workgroups) split into --amr-passes passes."""
    case = I.config3()
    tr = case.tree
    grid = api.Grid(torch.as_tensor(case.phi.astype(np.float32), device=dev), case.box,
                    n_base=tr.n, child_oct=torch.as_tensor(tr.child_oct, device=dev),
                    max_level=tr.max_level)
    tens = api.TidalTensor(grid, "fp32").build(grid)
    plan = api.Plan()
    b = I.config3_rays(args.amr_rays)
    gb = [api.RayBundle(torch.as_tensor(b.dirs, device=dev), b.nx, b.ny, b.chi_s, b.chi_hi,
                        b.chi_lo)]
    plan.set_shape(gb, persistent=0, block=256, passes=args.amr_passes)
    nr = b.nx * b.ny
    kap = torch.zeros(nr, dtype=torch.float32, device=dev)
    comp = torch.zeros(nr, dtype=torch.float32, device=dev)
    ms = []
    for _ in range(2):
        kap.zero_()
        comp.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.trace(plan, tens, gb, case.observer, kappa=kap, kappa_comp=comp, persistent=-1)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
        log(f"AMR map, {args.amr_passes} passes: {ms[-1]:.1f} ms")
    return {"amr_profile": {"passes": args.amr_passes, "ms": ms, "cells": int(tr.n_cells)}}


def host_cpu():
    """Model name, sockets and the cores this process may run on (the oracle's
    OpenMP threads), from /proc/cpuinfo and the scheduler affinity."""
    model, sockets = "unknown", set()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name") and model == "unknown":
                model = line.split(":", 1)[1].strip()
            elif line.startswith("physical id"):
                sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        cores = min(cores, int(omp))
    return model, max(len(sockets), 1), max(int(cores or 1), 1)


def batched_profile(args, api, I, torch, dev):
    """The 64 batched bundles alone, for profilers: one tensor build of the AMR
    tree and --profile-reps persistent launches of all bundles in the shape the
    tuner picks for them (16 wavefronts per CU, 16 passes)."""
    case = I.config3()
    tr = case.tree
    grid = api.Grid(torch.as_tensor(case.phi.astype(np.float32), device=dev), case.box,
                    n_base=tr.n, child_oct=torch.as_tensor(tr.child_oct, device=dev),
                    max_level=tr.max_level)
    tens = api.TidalTensor(grid, "fp32").build(grid)
    plan = api.Plan()
    bundles, offset = [], 0
    for s in I.config4_specs():
        bb = I.bundle_from_spec(s)
        bundles.append(api.RayBundle(torch.as_tensor(bb.dirs, device=dev), bb.nx, bb.ny,
                                     bb.chi_s, bb.chi_hi, bb.chi_lo, offset))
        offset += bb.nx * bb.ny
    plan.set_shape(bundles, persistent=1, waves_per_cu=16, passes=args.amr_passes)
    kap = torch.zeros(offset, dtype=torch.float32, device=dev)
    comp = torch.zeros(offset, dtype=torch.float32, device=dev)
    ms = []
    for _ in range(args.profile_reps):
        kap.zero_()
        comp.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.trace(plan, tens, bundles, case.observer, kappa=kap, kappa_comp=comp, persistent=-1)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
        log(f"batched bundles, {args.amr_passes} passes: {ms[-1]:.1f} ms")
    return {"batched_profile": {"passes": args.amr_passes, "ms": ms, "rays": offset}}


def adjoint_profile(args, api, I, torch, dev):
    """The adjoint configuration alone, for profilers: --profile-reps forward and
    backward steps (tensor build, march, scatter and transpose)."""
    args.steps, args.warmup = args.profile_reps, 0
    return {"adjoint_profile": adjoint_leg(args, api, I, torch, dev)}


def cpu_baseline(ctx, results, target_s):
    """FP64 oracle on the host over the whole light cone (every segment with
    its own vertex tensor) for a deterministic ray sample, on all the cores
    this process may use, and on one thread for a smaller sample; the GPU's
    crossing hashes and counts of the sampled rays (from the full-map launch
    with hashes) are compared with the oracle's in every segment."""
    from oracle import oracle as O
    phis, segs, dirs = ctx["phis"], ctx["segs"], ctx["dirs"]
    n, box, obs, chi_s = ctx["n"], ctx["box"], ctx["obs"], ctx["chi_s"]
    model, sockets, cores = host_cpu()
    r32 = results["fp32"]
    per_ray = r32["cross"] / dirs.shape[0]
    # sample size for about target_s of tracing at ~1e7 crossings/s per core
    want = int(min(dirs.shape[0], max(4096, target_s * 1.0e7 * cores / per_ray)))
    rng = np.random.default_rng(12345)
    sel = np.sort(rng.choice(dirs.shape[0], size=want, replace=False))
    # one-thread sample: every 64th ray of the sample's first 1/8 (a few seconds)
    one = sel[: max(64, want // 8)][::64]
    kap = np.zeros(want)
    t_tensor = t_trace = t_one = 0.0
    cross = cross_one = 0
    hash_ok = count_ok = True
    for k, (hi, lo, _) in enumerate(segs):
        phi = phis[k].double().cpu().numpy()
        t0 = time.perf_counter()
        tv = O.vertex_tensor(phi)
        t_tensor += time.perf_counter() - t0
        # one thread first: the oracle keeps the last thread count, and the
        # all-thread call below restores it for the next segment's tensor
        t0 = time.perf_counter()
        r1 = O.trace_uniform(n, box, obs, dirs[one], chi_s, hi, lo, tv=tv, threads=1)
        t_one += time.perf_counter() - t0
        t0 = time.perf_counter()
        r = O.trace_uniform(n, box, obs, dirs[sel], chi_s, hi, lo, tv=tv, threads=cores)
        t_trace += time.perf_counter() - t0
        cross_one += int(r1.ncross.sum())
        kap += r.kappa
        cross += int(r.ncross.sum())
        gh, gc = r32["seg_hash"][k]
        hash_ok &= bool(np.array_equal(gh.cpu().numpy().view(np.uint64)[sel], r.hash))
        count_ok &= bool(np.array_equal(gc.cpu().numpy()[sel], r.ncross))
        del tv
        log(f"oracle segment {k}: {int(r.ncross.sum())} crossings, hashes equal: {hash_ok}")
    log(f"oracle: {want} rays x {len(segs)} segments, {cross} crossings in {t_trace:.1f}s "
        f"(+{t_tensor:.1f}s tensors); one thread: {cross_one} crossings in {t_one:.1f}s")
    gk = r32["kappa"][sel]
    err = np.abs(gk - kap)
    lim = np.maximum(1e-5 * np.abs(kap), 1e-7)
    cb = {"value": cross / t_trace, "unit": "crossings/s", "cores": cores, "kind": "oracle",
          "sample": f"{want} of {dirs.shape[0]} rays through all {len(segs)} chi segments of "
                    f"the light cone ({cross} crossings); FP64 C oracle, OpenMP over rays on "
                    f"{cores} threads; its {len(segs)} vertex tensors ({n}^3 each) took "
                    f"{t_tensor:.1f}s, not included",
          "cpu_model": model, "sockets": sockets,
          "ns_per_crossing_one_thread": t_one / cross_one * 1e9,
          "one_thread_sample": f"{one.size} rays (every 64th of the sample's first eighth) "
                               f"through all {len(segs)} segments, {cross_one} crossings, "
                               "measured on one thread",
          "ns_per_crossing_per_core_derived": t_trace * cores / cross * 1e9,
          "ns_per_crossing_per_core_derived_note": "all-thread time x threads / crossings "
                                                  "(derived, not measured per core)"}
    par = {"rays": int(want), "kappa_max_err_over_tol": float(np.max(err / lim)),
           "crossing_hashes_equal": hash_ok, "crossing_counts_equal": count_ok,
           "segments": len(segs),
           "tolerance": "max(1e-5 |kappa|, 1e-7) per ray, FP32-Kahan GPU vs FP64 oracle; "
                        "crossing hashes and counts bit-exact in every segment"}
    return cb, par


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--rays", type=int, default=2048)
    ap.add_argument("--segments", type=int, default=20)
    ap.add_argument("--amr-rays", type=int, default=4096)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-amr", action="store_true")
    ap.add_argument("--no-method-a", action="store_true")
    ap.add_argument("--no-sources", action="store_true",
                    help="skip the ten-source-redshift light cone")
    ap.add_argument("--no-isw", action="store_true", help="skip the ISW light cone")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint configuration")
    ap.add_argument("--no-tune", action="store_true", help="skip the AMR leg's autotuning")
    ap.add_argument("--tune-lightcone", action="store_true",
                    help="autotune the light-cone launch shape per segment (default: one "
                         "wavefront per tile, 256-thread workgroups)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--profile-steps", action="store_true",
                    help="short light-cone-only run for profilers (no FP64, CPU or AMR legs)")
    ap.add_argument("--profile-amr", action="store_true",
                    help="AMR map only (for profilers): tensor build and two marches")
    ap.add_argument("--amr-passes", type=int, default=16,
                    help="passes of the --profile-amr and --profile-batched marches")
    ap.add_argument("--profile-batched", action="store_true",
                    help="the 64 batched bundles only (for profilers)")
    ap.add_argument("--profile-adjoint", action="store_true",
                    help="the adjoint configuration only (for profilers)")
    ap.add_argument("--profile-reps", type=int, default=2,
                    help="launches of the --profile-batched / --profile-adjoint modes")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the light cone, copy this many MiB device-to-device (a plain "
                         "copy kernel that calibrates the profiler's byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the tracer runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.profile_steps:
        args.no_fp64 = args.no_cpu = args.no_amr = args.no_method_a = args.no_sources = True
        args.no_isw = args.no_adjoint = True

    import torch
    from paper_1601_02012_amd import api, inputs as I

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile_amr:
        print(json.dumps(amr_profile(args, api, I, torch, dev)), flush=True)
        return
    if args.profile_batched:
        print(json.dumps(batched_profile(args, api, I, torch, dev)), flush=True)
        return
    if args.profile_adjoint:
        print(json.dumps(adjoint_profile(args, api, I, torch, dev)), flush=True)
        return
    results, ctx = lightcone_leg(args, api, I, torch, dev)
    r32 = results["fp32"]
    nseg = len(ctx["segs"])
    value = r32["cross"] / (r32["step_ms"] * 1e-3)
    march_launch_ms = r32["march_ms"] / nseg
    cross_per_launch = r32["cross"] / nseg
    bytes_gbs = BYTES_PER_CROSSING["fp32"] * cross_per_launch / (march_launch_ms * 1e-3) / 1e9
    flops_eq = FLOPS_PER_CROSSING["fp32"] + 2 * FLOPS_PER_CROSSING["fp64"]
    achieved = flops_eq * cross_per_launch / (march_launch_ms * 1e-3) / 1e12
    prof = profile_figures()
    traffic = prof.get("hbm_bytes_per_launch")
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
        "config": {"workload": f"light cone: uniform periodic {ctx['n']}^3 grid, box 1000 Mpc/h, "
                               f"FP32 lognormal potential, {args.rays}x{args.rays} rays over 5x5 "
                               f"deg, {nseg} chi segments to z=1, tensor rebuilt over the whole "
                               "grid every segment, FP32-Kahan march",
                   "grid": ctx["n"], "rays": args.rays ** 2, "segments": nseg,
                   "chi_s": ctx["chi_s"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "flops_per_crossing": {**FLOPS_PER_CROSSING, "fp32_equivalent": flops_eq},
                     "bytes_model": {"achieved": bytes_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                     "frac": bytes_gbs / PEAK_HBM_GBS},
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, "
                                     "copy-calibrated)",
                     "algorithmic_bytes_per_launch": BYTES_PER_CROSSING["fp32"] * cross_per_launch,
                     "measured_hbm_gbs": (traffic / (march_launch_ms * 1e-3) / 1e9
                                          if traffic else None),
                     "l2_hit_frac": prof.get("march_l2_hit_frac"),
                     "valu_busy_frac": prof.get("march_valu_busy_frac"),
                     "valu_insts_per_crossing": prof.get("march_valu_insts_per_crossing"),
                     "hw_fp32_flops_per_crossing": prof.get("march_hw_fp32_flops_per_crossing"),
                     "lane_utilisation": prof.get("march_lane_utilisation"),
                     "kernel": "march_uniform (FP32-Kahan)",
                     "bytes_per_crossing": BYTES_PER_CROSSING["fp32"],
                     "launch_ms": march_launch_ms, "crossings_per_launch": cross_per_launch,
                     "march_source": march_source_hash()},
        "march_crossings_per_s": r32["cross"] / (r32["march_ms"] * 1e-3),
        "tensor_build_ms_per_segment": r32["build_ms"] / nseg,
        "tensor_build_gbs": BYTES_PER_VERTEX["fp32"] * ctx["n"] ** 3
                            / (r32["build_ms"] / nseg * 1e-3) / 1e9,
        "tuned_shapes": sorted(set(r32["shapes"])),
        "all_rays_ok": r32["status_ok"],
    }
    if "method_a" in results:
        out["method_a"] = results["method_a"]
    if "sources" in results:
        out["many_sources"] = results["sources"]
    if "isw" in results:
        out["isw"] = results["isw"]
    if "adjoint" in results:
        out["adjoint"] = results["adjoint"]
    if "fp32_box" in results:
        rb = results["fp32_box"]
        box = {"value": rb["cross"] / (rb["step_ms"] * 1e-3), "unit": "crossings/s",
               "ms_per_step": rb["step_ms"],
               "tensor_build_ms_per_segment": rb["build_ms"] / nseg,
               "vertex_box_fraction_of_grid": rb["box_frac"],
               "kappa_bitwise_equal_to_whole_grid": bool(np.array_equal(rb["kappa"],
                                                                        r32["kappa"])),
               "note": "tensor rebuilt every segment only on the vertex box its rays read "
                       "(rr_rays_vertex_box, computed once per geometry)"}
        if "fp64_box" in results:
            box["speedup_vs_fp64_box"] = results["fp64_box"]["step_ms"] / rb["step_ms"]
        out["box_build"] = box
    if "fp64" in results:
        r64 = results["fp64"]
        out["fp64_crossings_per_s"] = r64["cross"] / (r64["step_ms"] * 1e-3)
        out["speedup_vs_fp64"] = r64["step_ms"] / r32["step_ms"]
        out["fp64_march_crossings_per_s"] = r64["cross"] / (r64["march_ms"] * 1e-3)
        out["fp64_tensor_build_ms_per_segment"] = r64["build_ms"] / nseg
        out["crossings_equal_fp32_fp64"] = r64["cross"] == r32["cross"]
        ref = r64["kappa"]
        err = np.abs(r32["kappa"] - ref)
        lim = np.maximum(1e-5 * np.abs(ref), 1e-7)
        out["kappa_fp32_vs_fp64"] = {"max_err_over_tol": float(np.max(err / lim)),
                                     "max_abs_err": float(err.max()),
                                     "rms_kappa": float(np.sqrt(np.mean(ref ** 2)))}
    if not args.no_cpu:
        out["cpu_baseline"], out["oracle_parity_sample"] = cpu_baseline(ctx, results,
                                                                        args.cpu_seconds)
    del ctx
    torch.cuda.empty_cache()
    if not args.no_amr:
        out.update(amr_leg(args, api, I, torch, dev))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
