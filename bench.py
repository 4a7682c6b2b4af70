"""Benchmark of the converted-view SPH step on one MI355X.

One step = cells_build, the density view (gather, density with the
smoothing-length iteration, scatter), the force view (gather, force, time-step
and conservation reduction, scatter) and kick_drift, all through the C-ABI on
one stream.  The workload (--workload, default kh256) is the largest
single-GPU configuration: the Kelvin-Helmholtz shear layer on a 256^3 lattice
(16,777,216 particles) in the periodic unit box, 256-byte records, FP64.

Before the timed runs the library's tuner picks, untimed, each loop's layout
and tile shape on the same records (with --tune-grid also the grid: cells per
support length 1, 2 or 3); the timed steps run with that choice (--no-tune:
SoA views).  The grid is otherwise the generated one (one cell spans the
support 2h with 10 % headroom).

value = (density pairs + force pairs) per second over the timed steps, the pairs
counted by the kernels themselves (j != i inside the support at the accepted h).
Besides the FP64 form the line carries the FP32 form on the same workload and
the batched form (FP32 pairs, graph-replayed steps) on the 2^20-particle
Plummer sphere, each with its speedup over the plain FP64 GPU form there.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# algorithmic flops per true pair (FMA = 2, sqrt and division = 1 each) of the
# density and the force formulas, per smoothing kernel: 31 and 75 for the cubic
# spline; the quartic's w and w' take 11 more per density pair, its w' 7 more
# per side of a force pair
FLOPS_DENSITY_PAIR = {"cubic": 31, "quartic": 42}
FLOPS_FORCE_PAIR = {"cubic": 75, "quartic": 89}
# algorithmic bytes per particle of each piece of the FP64 converted step:
# members read + members written (a density pass reads x, y, z, m, h and
# writes h, rho, omega, wcount; the force loop reads 12 members and writes 5)
BYTES_FP64 = {"density_gather": 40 + 40, "density_loop_pass": 40 + 32, "density_scatter": 32 + 32,
              "force_gather": 96 + 96, "force_loop": 96 + 40, "reduce": 48 + 40, "force_scatter": 40 + 40,
              "kick_drift": 120 + 88}
PEAK_FP64_VALU = 256 * 2.4e9 * 128          # 256 CUs x 2.4 GHz x 64 FMA lanes: 78.6 TFLOP/s
PEAK_FP32_VALU = 157.3e12                   # published, needs packed FP32
HBM_PEAK = 8.0e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


PAIR_SRC = os.path.join(ROOT, "paper_2502_16517_amd", "csrc", "k_pair.hip")
TRAFFIC_FILE = None     # the committed counter summary of the workload (set in main)


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"pair_loops_{workload}_fp64_counters.md")


def profiled_choice():
    """grid / density_layout / force_layout the committed counters were taken
    with, when they are for the current pair kernels; else None."""
    try:
        text = open(TRAFFIC_FILE).read()
        src = hashlib.sha256(open(PAIR_SRC, "rb").read()).hexdigest()[:16]
    except (OSError, TypeError):
        return None
    for line in text.splitlines():
        line = line.strip()
        if line.startswith("traffic:"):
            kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
            if kv.get("sha256/16") == src:
                return {k: kv.get(k) for k in ("grid", "density_layout", "force_layout")}
    return None


def kernel_variant(layout_name):
    """The pair kernel a layout runs: on the records (direct or sorted) or on a
    view, masked or branching (the FP64 kernels' template arguments)."""
    kind, _, mode = layout_name.split("/")
    return ("records" if kind in ("direct", "sorted") else "view", mode)


def measured_traffic(choice):
    """HBM bytes per launch of each pair loop from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (scaled by a plain copy's counters), for
    the loops whose kernel (source hash, grid, records or view, masked or
    branching) is the one the counters were taken on; with the layout they
    were taken with.  {} when none applies."""
    try:
        text = open(TRAFFIC_FILE).read()
        src = hashlib.sha256(open(PAIR_SRC, "rb").read()).hexdigest()[:16]
    except (OSError, TypeError):
        return {}
    for line in text.splitlines():
        line = line.strip()
        if not line.startswith("traffic:"):
            continue
        kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
        if kv.get("sha256/16") != src or kv.get("grid") != choice["grid"]:
            return {}
        out = {}
        for loop in ("density", "force"):
            prof = kv.get(loop + "_layout")
            if prof and kernel_variant(prof) == kernel_variant(choice[loop + "_layout"]):
                out[loop] = (float(kv[loop]), prof)
        return out
    return {}


# the synthetic workloads: generator, parameters other than the defaults, and
# what they are
WORKLOADS = {
    "tube64": ("config2", {}, "two-state tube 64^3 + 32^3 = 294,912 particles, periodic [0,2]x[0,1]^2"),
    "kh128": ("config3", {}, "Kelvin-Helmholtz shear layer 128^3 = 2,097,152 particles, periodic unit box"),
    "plummer1M": ("config4", {"headroom": 1.6},
                  "Plummer sphere a = 0.1 truncated at r = 1, 1,048,576 particles, open box [-1,1]^3, "
                  "cells of 0.02 (1 to ~2000 particles)"),
    "kh256": ("config5", {}, "Kelvin-Helmholtz shear layer 256^3 = 16,777,216 particles, periodic unit box"),
}
PKW = {}
HOST_RECORDS = False
# neighbour-list capacity of the list walks (the lattices' lists hold at most
# 81 entries, the Plummer sphere's about 60)
LIST_CAP = 128
# smoothing kernels (the library's kernel ids)
KERNELS = {"cubic": 0, "quartic": 1}


def make_stepper(torch, sv, inputs, w, precision, tuned=None, merged=False):
    """A Stepper on the workload; tuned = (grid, density layout, force layout);
    merged: one view over both loops with the density layout.  With
    HOST_RECORDS the records live in pinned host memory."""
    grid, ld, lf = tuned if tuned else (tuple(w.grid), sv.layout(), sv.layout())
    p = sv.params_init(w.lo, w.length, grid, w.periodic)
    p.eta = w.eta
    for k, v in PKW.items():
        setattr(p, k, v)
    if precision == sv.PREC_FP32:
        p.h_tol = 1e-6
    aos = None
    if HOST_RECORDS:
        import numpy as np
        aos = torch.from_numpy(inputs.as_bytes(np.ascontiguousarray(w.rec))).pin_memory()
    st = sv.Stepper(w.rec, p, precision, layout_density=ld, layout_force=lf,
                    stream=torch.cuda.current_stream(), merged=merged, aos=aos)
    return st


def tune(torch, sv, inputs, w, precision, tune_grid):
    """The tuner's choice for this workload: after two steps (valid force
    inputs), each loop's layout and tile shape over the built-in candidates;
    with tune_grid first the grid among cells per support 1, 2, 3 of the
    largest h.  Untimed set-up; the tables go to stderr."""
    st = make_stepper(torch, sv, inputs, w, precision)
    for _ in range(2):
        st.step()
    cps = None
    h_ref = None
    if tune_grid:
        cps = (1, 2, 3)
        h_ref = float(st.records()[:, inputs.SLOT["h"]].max())
    # the layouts the committed counters were taken with go first, so they win
    # ties with the others (candidates within 1.5 % of the fastest)
    cands = None
    prof = profiled_choice() if precision == sv.PREC_FP64 else None
    if prof and prof.get("density_layout") and prof.get("force_layout"):
        base = sv.autotune_candidates()
        cands = {}
        for key in ("density", "force"):
            first = layout_of(sv, prof[key + "_layout"])
            rest = [c for c in base if sv.layout_name(c) != sv.layout_name(first)]
            cands[key] = [first] + rest
    # between one bench run and the next the trial medians move by a few per
    # cent: the first candidate within 3 % of the fastest is taken (the force
    # loop is tuned after a density pass with the density layout so taken)
    res = st.autotune(candidates=cands, reps=5, cells_per_support=cps, h_ref=h_ref, within=0.03)
    grid = tuple(st.p.grid)
    ld, lf = st.ld, st.lf
    st.close()
    if tune_grid:
        log(f"[bench]   grid candidates (ms for cells_build + density + force): "
            + ", ".join(f"{'x'.join(map(str, g))} {ms:.3f}" for g, ms in res["grid"][1])
            + f" -> {'x'.join(map(str, grid))}")
    for key in ("density", "force"):
        best, table = res[key]
        top = sorted(table, key=lambda t: t[1])[:4]
        log(f"[bench]   {key}: " + ", ".join(f"{sv.layout_name(l)} {ms:.3f}" for l, ms in top)
            + f" -> {sv.layout_name(best)}")
    return grid, ld, lf


def layout_of(sv, name):
    """Inverse of sphview.layout_name: kind/tpiN|tpiauto/branch|masked."""
    kind, tpi, mode = name.split("/")
    kinds = {"soa": (sv.LAYOUT_SOA, 0), "direct": (sv.LAYOUT_DIRECT, 0), "sorted": (sv.LAYOUT_SORTED, 0)}
    k, wdt = kinds[kind] if kind in kinds else (sv.LAYOUT_AOSOA, int(kind[len("aosoa"):]))
    return sv.layout(k, wdt, tpi=0 if tpi == "tpiauto" else int(tpi[3:]), masked=1 if mode == "masked" else 0)


def choice_of(sv, tuned):
    grid, ld, lf = tuned
    return {"grid": "x".join(map(str, grid)), "density_layout": sv.layout_name(ld),
            "force_layout": sv.layout_name(lf)}


EVENTS = ("start", "built", "d_gathered", "d_loop", "d_scattered", "f_gathered", "f_loop", "reduced", "f_scattered",
          "kicked")


def run_timed(torch, sv, st, steps, warmup, graph=False):
    """Warm up, then time exactly `steps` steps; HIP events on the stream
    between the pieces of each step."""
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        st.step()
    torch.cuda.synchronize()
    g = None
    if graph:
        sv.graph_begin(s)
        st.step()
        g = sv.graph_end(s)
        torch.cuda.synchronize()
    before = st.read_state()
    ev = [{name: torch.cuda.Event(enable_timing=True) for name in EVENTS} for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e_start.record(s)
    for k in range(steps):
        if graph:
            sv.graph_launch(g, s)
            continue
        e = ev[k]
        e["start"].record(s)
        sv.begin_step(st.state, s)
        sv.cells_build(st.cells, st.aos, st.d_cells, st.state, s)
        e["built"].record(s)
        sv.aos_to_soa(st.v_dens, st.cells, s)
        e["d_gathered"].record(s)
        sv.sph_density(st.v_dens, st.cells, st.p, st.state, s)
        e["d_loop"].record(s)
        if not st.merged:              # one view over both loops: no scatter and gather between
            sv.soa_to_aos(st.v_dens, s)
        e["d_scattered"].record(s)
        if not st.merged:
            sv.aos_to_soa(st.v_force, st.cells, s)
        e["f_gathered"].record(s)
        sv.sph_force(st.v_force, st.cells, st.p, st.state, s)
        e["f_loop"].record(s)
        sv.step_reduce(st.v_force, st.p, st.state, s)
        e["reduced"].record(s)
        sv.soa_to_aos(st.v_force, s)
        e["f_scattered"].record(s)
        sv.kick_drift(st.aos, st.d_kick, st.n, st.p, st.state, s)
        e["kicked"].record(s)
    e_end.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    after = st.read_state()
    ms = e_start.elapsed_time(e_end)
    res = dict(ms_total=ms, wall_s=wall, pairs=after.pairs_total - before.pairs_total,
               flags=after.flags, state=after)
    if not graph:
        span = lambda a, b: sum(x[a].elapsed_time(x[b]) for x in ev) / steps
        res["ms_density"] = span("d_gathered", "d_loop")
        # the force loop with its windows from the converged h
        res["ms_force"] = span("f_gathered", "f_loop")
        # the span of the two views: first density gather to last force scatter
        res["ms_span"] = span("built", "f_scattered")
        for name, a, b in (("cells", "start", "built"), ("density_gather", "built", "d_gathered"), ("density_scatter", "d_loop", "d_scattered"),
                           ("force_gather", "d_scattered", "f_gathered"), ("force_scatter", "reduced", "f_scattered"),
                           ("kick_drift", "f_scattered", "kicked"), ("reduce", "f_loop", "reduced")):
            res["ms_" + name] = span(a, b)
        log("[bench]   per-step density ms " + " ".join(f"{x['d_gathered'].elapsed_time(x['d_loop']):.3f}" for x in ev))
        log("[bench]   per-step force ms   " + " ".join(f"{x['f_gathered'].elapsed_time(x['f_loop']):.3f}" for x in ev))
    if g is not None:
        sv.graph_destroy(g)
    return res


def run_whole_steps(torch, st, steps, warmup):
    """Warm up, then time exactly `steps` calls of the stepper's own step (its
    forms that the piecewise timing does not reproduce: overlapped prefetch,
    records reached by address); HIP events around the timed steps only."""
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        st.step()
    torch.cuda.synchronize()
    before = st.read_state()
    e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e_start.record(s)
    for _ in range(steps):
        st.step()
    e_end.record(s)
    torch.cuda.synchronize()
    after = st.read_state()
    return dict(ms_total=e_start.elapsed_time(e_end), pairs=after.pairs_total - before.pairs_total,
                flags=after.flags, state=after)


def pair_evals_per_step(torch, sv, st):
    """One more (untimed) step to read the per-step pair counters."""
    st.step()
    s = st.read_state()
    return s.pair_evals_density, s.pairs_force, s.pairs_density


def copy_bandwidth(torch, mib=1024, reps=5):
    """The HBM rate a plain device-to-device copy reaches (bytes read + bytes
    written per second, best of reps), beside the 8 TB/s of the specification."""
    src = torch.ones((mib << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    best = None
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        dst.copy_(src)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    rate = 2 * (mib << 20) / (best / 1e3)
    return {"GB/s": rate / 1e9, "frac_of_peak": rate / HBM_PEAK, "bytes": 2 * (mib << 20), "ms": best}


def cpu_model():
    name = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return name


def cpu_baseline(inputs, w, kernel=0, sample_single=200_000, sample_all=1_000_000, seed=16517):
    """The oracle (plain scalar C; OpenMP over its target particles) timed on
    the host cores, on a bounded sample of one step of the same workload,
    single-threaded and on every host thread.

    The sample is a contiguous run of target particles in record order (as
    one thread of a whole step walks them), starting at a seeded offset.  Per
    thread count: density with the smoothing-length iteration, then the force,
    at those targets; each call also builds the oracle's cell list over all N
    particles, a fixed cost timed on its own with a single target.  The step
    estimate is that fixed cost plus the per-target cost times N, and its pairs
    the sample's mean pairs per target times N.  The force reads, for every
    particle, h as recorded, rho = m eta^3 / h^3 (the state the iteration
    converges to) and omega = 1, so it does not depend on a density pass over
    all N."""
    import numpy as np

    from oracle import oracle as orc

    S = inputs.SLOT
    rec = w.rec
    n = w.n
    box = orc.box_of(w.lo, w.length, w.periodic)
    c = {k: np.ascontiguousarray(rec[:, S[k]]) for k in S if k not in inputs.INT_SLOTS}
    rho = c["m"] * w.eta ** 3 / c["h"] ** 3
    omega = np.ones(n)
    rng = np.random.Generator(np.random.PCG64(seed))

    def run(targets, nthreads):
        t0 = time.perf_counter()
        d = orc.density(c["x"], c["y"], c["z"], c["m"], c["h"], box, w.eta, nthreads=nthreads, kernel=kernel,
                        targets=targets)
        t1 = time.perf_counter()
        f = orc.force(c["x"], c["y"], c["z"], c["vx"], c["vy"], c["vz"], c["m"], c["h"], rho, omega, c["u"],
                      c["alpha"], box, inputs.GAMMA, nthreads=nthreads, kernel=kernel, targets=targets)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, int(d["count"].sum()) + int(f["count"].sum())

    out = {}
    for label, nthreads, size in (("single", 1, sample_single), ("all", orc.max_threads(), sample_all)):
        size = min(size, n)
        i0 = int(rng.integers(0, n - size + 1))
        targets = np.arange(i0, i0 + size, dtype=np.int64)
        fd, ff, _ = run(targets[:1], nthreads)
        td, tf, pairs = run(targets, nthreads)
        fixed = fd + ff
        per_target = max(td + tf - fixed, 1e-12) / size
        t_step = fixed + per_target * n
        pairs_step = pairs * n / size
        out[label] = {"value": pairs_step / t_step, "threads": nthreads, "targets": size, "first_target": i0,
                      "s_sample": td + tf, "s_fixed": fixed, "s_step_estimate": t_step,
                      "pairs_step_estimate": pairs_step}
    a = out["all"]
    return {"value": a["value"], "unit": "pairs/s", "cores": a["threads"], "kind": "oracle",
            "sample": (f"{a['targets']} and {out['single']['targets']} consecutive target particles of the "
                       f"{n}-particle workload (density with h iteration + force, pairs = density + force "
                       f"pairs), on {a['threads']} and 1 threads, extrapolated to one step: "
                       f"{a['s_step_estimate']:.1f} s and {out['single']['s_step_estimate']:.1f} s per step"),
            "single_thread": out["single"]["value"], "all_threads": out["all"],
            "single": out["single"], "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def scattered_records(torch, inputs, w, where, seed=5, spread=2):
    """The records at seeded, shuffled slots of a buffer `spread` times larger,
    in pinned host or device memory, and the device list of their addresses
    in particle order."""
    import numpy as np
    rng = np.random.default_rng(seed)
    slots = rng.permutation(spread * w.n)[:w.n]
    buf = np.zeros((spread * w.n, inputs.NSLOT), dtype=np.float64)
    buf[slots] = w.rec
    raw = torch.from_numpy(buf.view(np.uint8).reshape(-1))
    raw = raw.pin_memory() if where == "host" else raw.cuda()
    ptrs = torch.from_numpy((raw.data_ptr() + slots.astype(np.uint64) * inputs.STRIDE).astype(np.uint64)
                            .view(np.int64)).cuda()
    return raw, ptrs


def host_records(torch, sv, inputs, w, desc, args):
    """The step with the records in pinned host memory: views (gathered once
    per loop) against loops on the records (every candidate fetched across
    the host link); views whose force members are fetched while the density
    loop runs; views over records scattered through a pool and reached by an
    address list, in host and in device memory.  One JSON line; its value is
    host-link inclusive."""
    global HOST_RECORDS
    HOST_RECORDS = True
    lays = args.layouts.split(",") if args.layouts else ["soa/tpiauto/branch", "soa/tpiauto/branch"]
    runs = {}
    for name, names in (("views", lays), ("records", ["direct/tpiauto/branch", "direct/tpiauto/branch"]),
                        ("views_overlap", lays), ("views_pointers_host", lays), ("views_pointers_device", lays)):
        log(f"[bench] host records, {name}: {names}")
        tuned = (tuple(w.grid), layout_of(sv, names[0]), layout_of(sv, names[1]))
        if name in ("views", "records"):
            st = make_stepper(torch, sv, inputs, w, sv.PREC_FP64, tuned)
        else:
            p = sv.params_init(w.lo, w.length, tuned[0], w.periodic)
            p.eta = w.eta
            for k, v in PKW.items():
                setattr(p, k, v)
            kw = dict(layout_density=tuned[1], layout_force=tuned[2], stream=torch.cuda.current_stream())
            if name == "views_overlap":
                import numpy as np
                raw = torch.from_numpy(inputs.as_bytes(np.ascontiguousarray(w.rec))).pin_memory()
                st = sv.Stepper(None, p, sv.PREC_FP64, aos=raw, overlap=True, **kw)
            else:
                raw, ptrs = scattered_records(torch, inputs, w, "host" if name.endswith("host") else "device")
                st = sv.Stepper(None, p, sv.PREC_FP64, aos=raw, record_ptrs=ptrs, **kw)
        if name in ("views", "records"):
            r = run_timed(torch, sv, st, args.steps, args.warmup)
            runs[name] = {"layouts": names, "ms_per_step": r["ms_total"] / args.steps,
                          "value": r["pairs"] / (r["ms_total"] / 1e3), "ms_density": r["ms_density"],
                          "ms_force": r["ms_force"], "ms_density_gather": r["ms_density_gather"],
                          "ms_force_gather": r["ms_force_gather"], "ms_kick_drift": r["ms_kick_drift"],
                          "flags": r["flags"]}
        else:
            r = run_whole_steps(torch, st, args.steps, args.warmup)
            runs[name] = {"layouts": names, "ms_per_step": r["ms_total"] / args.steps,
                          "value": r["pairs"] / (r["ms_total"] / 1e3), "flags": r["flags"]}
        st.close()
    out = {"metric": "pair interactions/s (density+force incl. AoS<->SoA views), records in pinned host memory",
           "value": runs["views"]["value"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": runs["views"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": desc + ", 256-byte 32-slot records in pinned host memory, FP64", "n": w.n,
                      "records": "pinned host"},
           "host_records": runs,
           "views_speedup": runs["records"]["ms_per_step"] / runs["views"]["ms_per_step"],
           "overlap_speedup": runs["views"]["ms_per_step"] / runs["views_overlap"]["ms_per_step"]}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--kernel", default="cubic", choices=list(KERNELS),
                    help="smoothing kernel of the measured step: the cubic M4 spline, or the quartic M5 the "
                         "paper employs")
    ap.add_argument("--host-records", action="store_true",
                    help="records in pinned host memory (every record access crosses the host link): the step "
                         "with the views of --layouts (SoA without it) and with loops on the records; not the "
                         "headline, whose records are resident in HBM")
    ap.add_argument("--no-merged", action="store_true",
                    help="skip the extra timing of one view over both loops (the tuned layouts that are views)")
    ap.add_argument("--no-other-kernel", action="store_true",
                    help="skip the extra timing of the other smoothing kernel with the same layouts")
    ap.add_argument("--workload", default="kh256", choices=list(WORKLOADS),
                    help="kh256 (the largest configuration) is the headline; the others are the parity "
                         "workloads, for context")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the tuner: SoA views for both loops")
    ap.add_argument("--layouts", default=None,
                    help="DENSITY,FORCE layout names as the tuner prints them (e.g. direct/tpiauto/branch,"
                         "soa/tpiauto/branch): use these instead of tuning (profiling runs)")
    ap.add_argument("--tune-grid", action="store_true",
                    help="let the tuner pick the grid too (it times one snapshot of the particles; over the "
                         "timed steps the generated grid did better on this workload)")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the extra timing of the state kept in SoA across steps")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched form (FP32 pairs, graph replay) on the Plummer sphere")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--list-cap", type=int, default=0,
                    help="neighbour-list capacity per particle: > 0 runs both pair loops as list walks "
                         "(one lane per particle), 0 the item kernels over cell windows")
    ap.add_argument("--symmetric", action="store_true",
                    help="with --list-cap: the force loop evaluates each pair once (Newton's third law) and "
                         "stores the partner's side")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-traffic kernel for "
                         "scaling the profiler's FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md for how "
              "the step would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2502_16517_amd import inputs
    from paper_2502_16517_amd import sphview as sv

    torch.cuda.set_device(0)
    # one side stream (default priority) for everything: graph capture needs a
    # stream other than the legacy null stream, and events record on it
    torch.cuda.set_stream(torch.cuda.Stream())
    if args.calib_copy_mib:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mib} MiB done")
        del src, dst
    hbm_copy = None
    if not args.calib_copy_mib:
        hbm_copy = copy_bandwidth(torch)
        log(f"[bench] device copy: {hbm_copy['GB/s']:.0f} GB/s (read + write)")
    global TRAFFIC_FILE
    TRAFFIC_FILE = traffic_file(args.workload)
    gen, pkw, desc = WORKLOADS[args.workload]
    PKW.update(pkw)
    PKW["kernel"] = KERNELS[args.kernel]
    PKW["list_cap"] = args.list_cap
    PKW["symmetric"] = 1 if args.symmetric else 0
    log(f"[bench] generating the workload: {desc}")
    w = getattr(inputs, gen)()
    if args.host_records:
        host_records(torch, sv, inputs, w, desc, args)
        return
    if args.layouts:
        names = args.layouts.split(",")
        t64 = (tuple(w.grid), layout_of(sv, names[0]), layout_of(sv, names[1]))
    elif args.no_tune:
        t64 = (tuple(w.grid), sv.layout(), sv.layout())
    else:
        log("[bench] tuning fp64 (untimed)")
        t64 = tune(torch, sv, inputs, w, sv.PREC_FP64, args.tune_grid)

    log("[bench] fp64 eager")
    st = make_stepper(torch, sv, inputs, w, sv.PREC_FP64, t64)
    r64 = run_timed(torch, sv, st, args.steps, args.warmup)
    evals_d, pairs_f, pairs_d = pair_evals_per_step(torch, sv, st)
    st.close()
    if r64["flags"]:
        log(f"[bench] warning: status flags {r64['flags']:#x}")

    log("[bench] fp64 graph")
    st = make_stepper(torch, sv, inputs, w, sv.PREC_FP64, t64)
    g64 = run_timed(torch, sv, st, args.steps, args.warmup, graph=True)
    st.close()

    merged = None
    if not args.no_merged:
        # one view over both loops, with each tuned layout that is a view
        cands = []
        for lay in (t64[1], t64[2]):
            if lay.kind in (sv.LAYOUT_DIRECT, sv.LAYOUT_SORTED):
                continue
            if not any(sv.layout_name(lay) == sv.layout_name(c) for c in cands):
                cands.append(lay)
        for lay in cands:
            log(f"[bench] fp64 eager, one view over both loops, {sv.layout_name(lay)}")
            st = make_stepper(torch, sv, inputs, w, sv.PREC_FP64, (t64[0], lay, lay), merged=True)
            rm = run_timed(torch, sv, st, args.steps, args.warmup)
            st.close()
            rec = {"layout": sv.layout_name(lay), "value": rm["pairs"] / (rm["ms_total"] / 1e3),
                   "ms_per_step": rm["ms_total"] / args.steps, "ms_span": rm["ms_span"],
                   "ms_gather": rm["ms_density_gather"], "ms_scatter": rm["ms_force_scatter"],
                   "ms_density": rm["ms_density"], "ms_force": rm["ms_force"], "flags": rm["flags"]}
            if merged is None or rec["value"] > merged["value"]:
                merged = rec

    other = None
    if not args.no_other_kernel:
        oname = next(k for k in KERNELS if k != args.kernel)
        log(f"[bench] fp64 eager, {oname} kernel, same layouts")
        PKW["kernel"] = KERNELS[oname]
        st = make_stepper(torch, sv, inputs, w, sv.PREC_FP64, t64)
        ro = run_timed(torch, sv, st, args.steps, args.warmup)
        st.close()
        PKW["kernel"] = KERNELS[args.kernel]
        other = {"kernel": oname, "value": ro["pairs"] / (ro["ms_total"] / 1e3),
                 "ms_per_step": ro["ms_total"] / args.steps, "ms_density": ro["ms_density"],
                 "ms_force": ro["ms_force"], "flags": ro["flags"]}

    f32 = None
    if not args.no_fp32:
        if args.no_tune:
            t32 = (tuple(w.grid), sv.layout(), sv.layout())
        else:
            log("[bench] tuning fp32 (untimed)")
            t32 = tune(torch, sv, inputs, w, sv.PREC_FP32, args.tune_grid)
        log("[bench] fp32 eager")
        st = make_stepper(torch, sv, inputs, w, sv.PREC_FP32, t32)
        r32 = run_timed(torch, sv, st, args.steps, args.warmup)
        st.close()
        f32 = {"value": r32["pairs"] / (r32["ms_total"] / 1e3), "ms_per_step": r32["ms_total"] / args.steps,
               "choice": choice_of(sv, t32),
               "ms_density": r32["ms_density"], "ms_force": r32["ms_force"], "ms_span": r32["ms_span"],
               "speedup_vs_fp64": (r32["pairs"] / r32["ms_total"]) / (r64["pairs"] / r64["ms_total"])}

    ms_step = r64["ms_total"] / args.steps
    value = r64["pairs"] / (r64["ms_total"] / 1e3)
    n = w.n
    passes = evals_d / max(pairs_d, 1)          # density passes per particle, on average
    # dominant kernel: the larger of the two pair loops
    dens_flops = evals_d * FLOPS_DENSITY_PAIR[args.kernel]
    force_flops = pairs_f * FLOPS_FORCE_PAIR[args.kernel]
    if r64["ms_force"] >= r64["ms_density"]:
        kern, flops, ms_k = "force", force_flops, r64["ms_force"]
    else:
        kern, flops, ms_k = "density", dens_flops, r64["ms_density"]
    achieved = flops / (ms_k / 1e3) / 1e12
    choice = choice_of(sv, t64)
    # the committed counters are those of the item kernels
    tr = measured_traffic(choice) if args.kernel == "cubic" and args.list_cap == 0 else {}
    traffic, traffic_layout = tr.get(kern, (None, None))
    if args.list_cap == 0:
        form = f"fp64 pair loop, {choice[kern + '_layout']}"
    elif kern == "force" and args.symmetric:
        form = f"fp64 symmetric list walk, list_cap {args.list_cap}"
    else:
        form = f"fp64 list walk, list_cap {args.list_cap}"
    roofline = {"bound": "alu", "kernel": f"sph_{kern} ({form})",
                "achieved": achieved,
                "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s", "frac": achieved / (PEAK_FP64_VALU / 1e12),
                "traffic": traffic,
                # the counters' run used the same kernel; its layout, when another
                "traffic_layout": traffic_layout,
                "flops_per_pair": {"density": FLOPS_DENSITY_PAIR[args.kernel],
                                   "force": FLOPS_FORCE_PAIR[args.kernel]},
                "density": {"ms": r64["ms_density"], "tflops": dens_flops / (r64["ms_density"] / 1e3) / 1e12,
                            "pair_evals": evals_d},
                "force": {"ms": r64["ms_force"], "tflops": force_flops / (r64["ms_force"] / 1e3) / 1e12,
                          "pairs": pairs_f}}

    # conversions (the paper's prologue and epilogue) and kick_drift: algorithmic
    # bytes (members read + members written, per particle) over their event times
    conv = {}
    for name in ("density_gather", "density_scatter", "force_gather", "force_scatter", "kick_drift"):
        direct = (name.startswith("density") and t64[1].kind in (sv.LAYOUT_DIRECT, sv.LAYOUT_SORTED)) or \
                 (name.startswith("force") and t64[2].kind in (sv.LAYOUT_DIRECT, sv.LAYOUT_SORTED))
        ms = r64["ms_" + name]
        per = BYTES_FP64[name]
        conv[name] = {"ms": ms, "bytes": 0 if direct and name != "kick_drift" else per * n,
                      "GB/s": None if direct and name != "kick_drift" else per * n / (ms / 1e3) / 1e9}
        if conv[name]["GB/s"] is not None:
            conv[name]["hbm_frac"] = conv[name]["GB/s"] * 1e9 / HBM_PEAK

    # lower bound of each piece of the span: max(algorithmic bytes / HBM peak,
    # algorithmic flops / FP64 vector peak); the fraction reported is
    # T_lower / T_measured, per piece and for the span (conversions, both
    # loops with every density pass, the step reduction)
    def t_lower(nbytes, nflops=0.0):
        return max(nbytes / HBM_PEAK, nflops / PEAK_FP64_VALU) * 1e3
    pieces = {
        "density_gather": (t_lower(n * BYTES_FP64["density_gather"]), r64["ms_density_gather"]),
        "density_loop": (t_lower(n * BYTES_FP64["density_loop_pass"] * passes, dens_flops), r64["ms_density"]),
        "density_scatter": (t_lower(n * BYTES_FP64["density_scatter"]), r64["ms_density_scatter"]),
        "force_gather": (t_lower(n * BYTES_FP64["force_gather"]), r64["ms_force_gather"]),
        "force_loop": (t_lower(n * BYTES_FP64["force_loop"], force_flops), r64["ms_force"]),
        "reduce": (t_lower(n * BYTES_FP64["reduce"]), r64["ms_reduce"]),
        "force_scatter": (t_lower(n * BYTES_FP64["force_scatter"]), r64["ms_force_scatter"]),
    }
    d4 = {k: {"t_lower_ms": lo, "t_ms": t, "frac": lo / t if t > 0 else None} for k, (lo, t) in pieces.items()}
    span_lower = sum(lo for lo, _ in pieces.values())
    d4["span"] = {"t_lower_ms": span_lower, "t_ms": r64["ms_span"], "frac": span_lower / r64["ms_span"]}
    d4["kick_drift"] = {"t_lower_ms": t_lower(n * BYTES_FP64["kick_drift"]), "t_ms": r64["ms_kick_drift"],
                        "frac": t_lower(n * BYTES_FP64["kick_drift"]) / r64["ms_kick_drift"]}

    persistent = None
    if not args.no_persistent:
        log("[bench] fp64 eager, state kept in SoA across steps")
        persistent = persistent_form(torch, sv, inputs, w, args)
        persistent["speedup_vs_views"] = ms_step / persistent["ms_per_step"]

    batched = None
    if not args.no_batched:
        batched = batched_form(torch, sv, inputs, args)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle, sampled)")
        cpu = cpu_baseline(inputs, w, KERNELS[args.kernel])

    out = {
        "metric": "pair interactions/s (density+force incl. AoS<->SoA views)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc + ", 256-byte 32-slot records, FP64",
                   "name": args.workload,
                   "n": w.n, "grid": list(t64[0]), "tuned": not (args.no_tune or args.layouts),
                   "kernel": args.kernel,
                   "layout": {"density": choice["density_layout"], "force": choice["force_layout"]},
                   "pairs_per_step": {"density": pairs_d, "density_all_passes": evals_d, "force": pairs_f}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "t_lower_over_t": d4,
        "graph": {"value": g64["pairs"] / (g64["ms_total"] / 1e3), "ms_per_step": g64["ms_total"] / args.steps},
        # pairs/s over the two views alone (gathers, loops, reduction, scatters),
        # without cells_build and kick_drift
        "span": {"value": r64["pairs"] / args.steps / (r64["ms_span"] / 1e3), "ms": r64["ms_span"]},
        "fp32": f32,
        "batched": batched,
        "other_kernel": other,
        # one view over both loops (gather before density, scatter after the reduction)
        "merged_view": merged,
        # the state in SoA across steps: no conversion inside a step
        "persistent_state": persistent,
        "conversions": conv,
        "reduce_ms": r64["ms_reduce"],
        "cells_build_ms": r64["ms_cells"],
        "hbm_frac_step": None,
        "hbm_copy": hbm_copy,
    }
    # whole-step HBM fraction: algorithmic view bytes (gathers, scatters, loop
    # inputs and outputs) over the step time
    algo_bytes = n * (BYTES_FP64["density_gather"] + BYTES_FP64["density_scatter"] + BYTES_FP64["force_gather"] +
                      BYTES_FP64["force_scatter"] + BYTES_FP64["density_loop_pass"] * passes +
                      BYTES_FP64["force_loop"])
    out["hbm_frac_step"] = algo_bytes / (ms_step / 1e3) / HBM_PEAK
    out["hbm_frac_span"] = algo_bytes / (r64["ms_span"] / 1e3) / HBM_PEAK
    print(json.dumps(out), flush=True)


def persistent_form(torch, sv, inputs, w, args):
    """The state kept in SoA across loops and steps (PersistentStepper): one
    gather of every physics member before the timed steps, then per step
    cells_build on the storage, the density and force loops directly on it
    (through the cells' perm, no copy), the step reduction and kick_drift on
    it.  The records are written back after the timed steps."""
    s = torch.cuda.current_stream()
    p = sv.params_init(w.lo, w.length, tuple(w.grid), w.periodic)
    p.eta = w.eta
    for k, v in PKW.items():
        setattr(p, k, v)
    st = sv.PersistentStepper(w.rec, p, stream=s)
    for _ in range(args.warmup):
        st.step()
    torch.cuda.synchronize()
    before = st.read_state()
    names = ("start", "built", "dens", "force", "kicked")
    ev = [{k: torch.cuda.Event(enable_timing=True) for k in names} for _ in range(args.steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for k in range(args.steps):
        e = ev[k]
        e["start"].record(s)
        st.build()
        e["built"].record(s)
        st.density()
        e["dens"].record(s)
        st.force()
        e["force"].record(s)
        st.kick()
        e["kicked"].record(s)
    e1.record(s)
    torch.cuda.synchronize()
    after = st.read_state()
    st.close()
    ms = e0.elapsed_time(e1)
    span = lambda a, b: sum(x[a].elapsed_time(x[b]) for x in ev) / args.steps
    return {"value": (after.pairs_total - before.pairs_total) / (ms / 1e3), "ms_per_step": ms / args.steps,
            "ms_cells": span("start", "built"), "ms_density": span("built", "dens"),
            "ms_force_and_reduce": span("dens", "force"), "ms_kick_drift": span("force", "kicked"),
            "layout": "direct on the SoA state (no per-loop copy)", "flags": after.flags,
            "conversion_bytes_per_step": 0,
            "open_close_bytes": 2 * 22 * 8 * w.n}


def batched_form(torch, sv, inputs, args):
    """The batching form on the 2^20-particle Plummer sphere (cells of 1 to
    ~2000 particles, dense cells ordered by sub-cell): neighbour-list walks
    that skip cells and 64-particle runs out of reach, FP32 pairs, the whole
    step replayed as one HIP graph; against the plain FP64 GPU form (the item
    kernels over cell windows, eager) on the same records, and the FP64 list
    walks.  SoA views (no tuning: a trial there costs a step)."""
    gen, pkw, desc = WORKLOADS["plummer1M"]
    saved = dict(PKW)
    PKW.clear()
    PKW.update(pkw)
    PKW["kernel"] = KERNELS[args.kernel]
    log(f"[bench] batched form: {desc}")
    w = getattr(inputs, gen)()
    lay = (tuple(w.grid), sv.layout(), sv.layout())
    steps, warm = args.batched_steps, 2
    runs = {}
    for name, prec, cap, graph in (("fp64_items_eager", sv.PREC_FP64, 0, False),
                                   ("fp64_lists_eager", sv.PREC_FP64, LIST_CAP, False),
                                   ("fp32_lists_graph", sv.PREC_FP32, LIST_CAP, True)):
        log(f"[bench]   {name}")
        PKW["list_cap"] = cap
        st = make_stepper(torch, sv, inputs, w, prec, lay)
        r = run_timed(torch, sv, st, steps, warm, graph=graph)
        st.close()
        runs[name] = {"value": r["pairs"] / (r["ms_total"] / 1e3), "ms_per_step": r["ms_total"] / steps,
                      "flags": r["flags"]}
        if not graph:
            runs[name].update(ms_density=r["ms_density"], ms_force=r["ms_force"], ms_cells=r["ms_cells"])
    PKW.clear()
    PKW.update(saved)
    b = runs["fp32_lists_graph"]
    base = runs["fp64_items_eager"]
    return {"workload": "plummer1M", "n": w.n, "steps": steps, "layout": "soa, list walks (cap %d)" % LIST_CAP,
            "value": b["value"], "ms_per_step": b["ms_per_step"], "flags": b["flags"],
            "fp64_eager": base, "fp64_lists_eager": runs["fp64_lists_eager"],
            "speedup_vs_fp64": b["value"] / base["value"],
            "speedup_lists_fp64_vs_items_fp64": runs["fp64_lists_eager"]["value"] / base["value"]}


if __name__ == "__main__":
    main()
