"""Benchmark: STTSV hyperedges/s on one MI355X, plus the H-eigenvector solve.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (default): the Zipf / power-law hypergraph, n = 1e6 vertices,
m = 5e6 edges, sizes P(k) ~ k^-2.5 on [2, 25], tensor order r = 25, Zipf(1.0)
membership, x uniform on (0, 1] -- seeded synthetic data.  A step is one full
STTSV y = B x^(r-1) (every edge-kernel launch plus the node reduction) with
x and y resident in HBM.  Prints one JSON line.
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
PEAK_FP64_VALU = 78.6e12   # FLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
PEAK_FP32_VALU = 157.3e12  # FLOP/s published (needs packed FP32, which this build disables)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def edge_fma(k, r):
    """Series FMAs of one edge of size k at order r, as the kernels compute
    them: truncated products W(W-1)/2 each, dot products of W terms."""
    W = r - k + 1
    prod = W * (W - 1) // 2
    if k == 1:
        return 0
    if k == 2:
        return max(W - 1, 0)
    if k == 3:
        return 2 * W + prod + max(W - 1, 0)
    return 2 * (k - 3) * prod + (k + 1) * W - 1


def stage_table(plan, xd, yd, prec, reps):
    from paper_2311_08595_amd import _lib
    lib = _lib.load()
    cap = 256
    ns = ctypes.c_int32()
    kinds = (ctypes.c_int32 * cap)()
    sizes = (ctypes.c_int32 * cap)()
    counts = (ctypes.c_int64 * cap)()
    ms = (ctypes.c_float * cap)()
    acc = None
    for _ in range(reps):
        _lib.check(lib.sttsv_apply_timed(plan._h, ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(yd.data_ptr()),
                                         _lib.PREC[prec], cap, ctypes.byref(ns), kinds, sizes, counts, ms))
        cur = np.array(ms[:ns.value], dtype=np.float64)
        acc = cur if acc is None else acc + cur
    acc /= reps
    return [dict(kind=int(kinds[i]), size=int(sizes[i]), count=int(counts[i]), ms=float(acc[i]))
            for i in range(ns.value)]


GEN_LO = [1, 9, 17, 25, 33, 41, 49, 57]
GEN_HI = [8, 16, 24, 32, 40, 48, 56, 63]


def stage_work(stages, bucket_k, bucket_m, r, bucket_l=None, prec="fp64", bucket_s=None):
    """Algorithmic FLOPs and HBM bytes of every stage.  Edge stages: series
    FMAs x 2 and 20 B per incidence (member id, gathered x, contribution);
    fused generic stages: the same summed over the buckets that no per-bucket
    stage covers and whose window is in the stage's range; the copy of x into
    degree-rank order: 4 B index + 8 B read + 8 B written per vertex;
    reduction levels: per term the value read (8 B, plus its 2 B LDS slot at
    level 0), per chunk its 12 B descriptor and the 8 B result.  An FP32
    apply runs compact: 12 B per incidence (4 B id, FP32 x, 32-bit
    contribution), 4 B more per vertex for the FP32 copy of x, and 4 B per
    level-0 term read.  Fused launches (kinds 1, 5, 6: one-lane generic kernel
    with its suffix stacks in LDS / in global memory / without stacks, whose
    extra series products are not counted; 4: lane groups) cover the
    buckets that no per-bucket stage covers, whose window is in the stage's
    range and whose kernel and stack placement match (bucket_s: the plan's
    stack flags).  Each entry: (FLOPs, bytes, description, launch threads or
    None)."""
    compact = prec == "fp32"
    sbit = 1 if prec == "fp64" else 2
    inc_b = 12.0 if compact else 20.0
    per_bucket = {s["size"] for s in stages if s["kind"] == 0}
    if bucket_l is None:
        bucket_l = [0] * len(bucket_k)
    out = []
    def kind_of(lanes, stack):
        if lanes > 0:
            return 4
        if bucket_s is not None and stack & (sbit << 2):
            return 6
        return 1 if bucket_s is None or stack & sbit else 5
    for s in stages:
        if s["kind"] == 0:
            k, m = s["size"], s["count"]
            out.append((2.0 * edge_fma(k, r) * m, inc_b * k * m, "edge k=%d (W=%d), %d edges" % (k, r - k + 1, m),
                        None))
        elif s["kind"] in (1, 4, 5, 6):
            g = s["size"]
            f = b = 0.0
            threads = 0
            stacks = bucket_s if bucket_s is not None else [0] * len(bucket_k)
            for k, m, lanes, st_ in zip(bucket_k, bucket_m, bucket_l, stacks):
                W = r - k + 1
                if (k >= 4 and k not in per_bucket and GEN_LO[g] <= W <= GEN_HI[g]
                        and kind_of(lanes, st_) == s["kind"]):
                    f += 2.0 * edge_fma(k, r) * m
                    b += inc_b * k * m
                    threads += 64 * ((m + 63) // 64) if lanes == 0 else 256 * ((m * lanes + 255) // 256)
            what = {1: "generic", 5: "generic (global-memory stacks)", 6: "generic (no stacks)",
                    4: "lane-group"}[s["kind"]]
            out.append((f, b, "%s edges W in [%d,%d], %d edges" % (what, GEN_LO[g], GEN_HI[g], s["count"]),
                        threads))
        elif s["kind"] == 3:
            out.append((0.0, (24.0 if compact else 20.0) * s["count"], "x into degree-rank order, n=%d" % s["count"],
                        None))
        else:
            per_term = (6.0 if compact else 10.0) if s["size"] == 0 else 8.0
            out.append((0.0, per_term * s["in_len"] + 20.0 * s["count"],
                        "reduce level %d, %d chunks" % (s["size"], s["count"]), None))
    return out


STTSV_SOURCES = ("edge_", "apply.hip", "reduce.hip", "internal.hpp", "plan.cpp")


def source_fingerprint():
    """sha256 over the sources of the STTSV kernels and the layout they run
    on: traffic figures taken from counters apply only while it is unchanged."""
    import hashlib
    d = os.path.join(ROOT, "paper_2311_08595_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.startswith(STTSV_SOURCES) and f.endswith((".hip", ".inc", ".hpp", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


PROFILE_STEMS = {"zipf": "sttsv_zipf_n1e6_m5e6_r25", "heavy": "sttsv_heavytail_n2e5_m2e6_r50"}


def _profile_rows(workload, kind, ncells, value_cells):
    """Rows {(kernel, grid or None): [values]} of a committed counter summary
    (profiles/<workload>_<kind>.md), or None when it is missing or was taken
    on other kernel sources (its fingerprint differs)."""
    path = os.path.join(ROOT, "profiles", "%s_%s.md" % (PROFILE_STEMS.get(workload, "-"), kind))
    if not os.path.exists(path):
        return None
    fp = None
    rows = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("source fingerprint:"):
                fp = line.split(":", 1)[1].strip().strip("`")
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            if len(cells) == ncells and (cells[1].isdigit() or cells[1] == "-"):
                try:
                    rows[(cells[0], int(cells[1]) if cells[1] != "-" else None)] = [float(cells[i])
                                                                                      for i in value_cells]
                except ValueError:
                    pass
    return rows if fp == source_fingerprint() else None


def _lookup(rows, kernel, grid):
    if rows is None:
        return None
    v = rows.get((kernel, grid))
    return v if v is not None else rows.get((kernel, None))


def measured_traffic(kernel, grid, workload="zipf"):
    """Calibrated HBM bytes per dispatch of (kernel, grid) from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None (no summary for this kernel, or
    the sources changed since the counters were taken)."""
    v = _lookup(_profile_rows(workload, "traffic", 6, [5]), kernel, grid)
    return None if v is None else v[0] * 1e6


def measured_valu(kernel, grid, workload="zipf"):
    """VALU and occupancy counters of (kernel, grid) from the committed
    summary (or None): wave count, FP64 and FP32 FMA wave-instructions,
    VALUBusy %, occupancy % and mean resident waves per CU."""
    v = _lookup(_profile_rows(workload, "valu_occupancy", 13, [3, 7, 8, 10, 11, 12]), kernel, grid)
    if v is None:
        return None
    return dict(waves=v[0], fma64_instr=v[1], fma32_instr=v[2], valu_busy_pct=v[3], occupancy_pct=v[4],
                waves_per_cu=v[5])


SMALL_KIND = {2: 0, 3: 1, 4: 2, 5: 3, 6: 4, 7: 5}


def stage_kernel(s, prec, r, threads=None):
    """Kernel name (template form, as the profiler prints it) and grid size
    of a stage; grid None where one launch per apply has that name.  FP32
    applies run the compact variants (template flag true; the workloads with
    committed counters have no FP64-fallback size under FP32)."""
    t, cp = ("double", "false") if prec == "fp64" else ("float", "true")
    if s["kind"] == 0 and s["size"] in SMALL_KIND:
        return ("edge_small<%s, %d, %d, %s>" % (t, r - s["size"] + 1, SMALL_KIND[s["size"]], cp),
                (s["count"] + 255) // 256 * 256)
    if s["kind"] in (1, 5, 6):   # launches of one range share the name: the grid tells them apart
        return "edge_generic<%s, %d, %d, %s>" % (t, GEN_LO[s["size"]], GEN_HI[s["size"]], cp), threads
    if s["kind"] == 4:
        return "edge_coop<%s, %d, %d, %s>" % (t, GEN_LO[s["size"]], GEN_HI[s["size"]], cp), threads
    if s["kind"] == 2:
        if s["size"] == 0:
            return "reduce_level0<%s>" % ("double" if prec == "fp64" else "unsigned int"), None
        return "reduce_level<false, double>", s["count"] * 8
    if s["kind"] == 3:
        return "permute_x", (s["count"] + 255) // 256 * 256
    return None, None


def roofline_of(stages, work, prec, r, workload=None):
    """Dominant stage and its roofline figures; with a workload whose counter
    summaries are committed, also the measured traffic and VALU counters of
    the dominant kernel."""
    i = max(range(len(stages)), key=lambda j: stages[j]["ms"])
    t = stages[i]["ms"] * 1e-3
    flops, byts, name, threads = work[i]
    peak_f = PEAK_FP64_VALU      # FP64 FMA and non-packed FP32 FMA issue at the same rate
    kname, grid = stage_kernel(stages[i], prec, r, threads)
    traffic = measured_traffic(kname, grid, workload) if kname and workload else None
    if flops / peak_f >= byts / PEAK_HBM:
        roof = dict(bound="alu", achieved=flops / t / 1e12, peak=peak_f / 1e12, unit="TFLOP/s",
                    frac=(flops / t) / peak_f, traffic=traffic, kernel=name, profiled_kernel=kname)
    else:
        roof = dict(bound="hbm", achieved=byts / t / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                    frac=(byts / t) / PEAK_HBM, traffic=traffic, kernel=name, profiled_kernel=kname,
                    algorithmic_bytes=byts)
    cnt = measured_valu(kname, grid, workload) if kname and workload else None
    if cnt is not None:
        # FMA wave-instructions x 64 lanes x 2: the issued FLOPs (masked lanes
        # included), over this run's kernel time, against the same peak
        issued = (cnt["fma64_instr"] + cnt["fma32_instr"]) * 128.0
        cnt["issued_flop"] = issued
        cnt["issued_frac"] = issued / t / peak_f
        roof["counters"] = cnt
    return stages[i], roof


def _oracle_terms(args):
    """Worker: the oracle's Alg. 2 terms of one contiguous range of edges."""
    from oracle import sttsv_ref
    eptr, eidx, n, r, x = args
    return sttsv_ref.incidence_terms(eptr, eidx, n, r, x)


def oracle_sttsv_parallel(eptr, eidx, n, r, x, procs):
    """The FP64 oracle (Alg. 2 terms + correctly rounded per-vertex sums)
    with its edges split into ``procs`` contiguous ranges computed by worker
    processes; the parent sums every vertex's terms with math.fsum, so the
    result is bitwise the oracle's serial one (fsum is correctly rounded)."""
    import multiprocessing as mp
    m = len(eptr) - 1
    cuts = np.linspace(0, m, procs + 1).astype(np.int64)
    jobs = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b > a:
            ep = eptr[a:b + 1] - eptr[a]
            jobs.append((ep, eidx[eptr[a]:eptr[b]], n, r, x))
    if procs > 1:
        with mp.get_context("fork").Pool(len(jobs)) as pool:
            parts = pool.map(_oracle_terms, jobs)
    else:
        parts = [_oracle_terms(j) for j in jobs]
    verts = np.concatenate([p[0] for p in parts])
    terms = np.concatenate([p[1] for p in parts])
    order = np.argsort(verts, kind="stable")
    vs, ts = verts[order], terms[order]
    bounds = np.searchsorted(vs, np.arange(n + 1))
    y = np.zeros(n)
    for v in np.flatnonzero(np.diff(bounds)):
        y[v] = math.fsum(ts[bounds[v]:bounds[v + 1]].tolist())
    return y


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def oracle_procs():
    # the GPU machine's CPU share is 16 threads per GPU, whatever os.cpu_count() shows
    return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline(w, sample_edges, procs, seed=0):
    rng = np.random.default_rng(seed)
    m = len(w["eptr"]) - 1
    pick = np.sort(rng.choice(m, size=min(sample_edges, m), replace=False))
    sizes = np.diff(w["eptr"])[pick]
    eptr = np.zeros(len(pick) + 1, dtype=np.int64)
    np.cumsum(sizes, out=eptr[1:])
    src = np.repeat(w["eptr"][pick], sizes) + (np.arange(eptr[-1]) - np.repeat(eptr[:-1], sizes))
    eidx = w["eidx"][src]
    t0 = time.perf_counter()
    oracle_sttsv_parallel(eptr, eidx, w["n"], w["r"], w["x"], procs)
    dt = time.perf_counter() - t0
    return dict(value=len(pick) / dt, unit="hyperedges/s", cores=procs, kind="oracle",
                cpu=host_cpu(),
                sample="%d random edges of the same hypergraph (all n=%d vertices), FP64 AAY terms in %d "
                       "worker processes over contiguous edge ranges, per-vertex fsum in the parent; %.1f s"
                       % (len(pick), w["n"], procs, dt))


def _timed_applies(plan, xd, yd, prec, warmup, reps):
    import torch
    for _ in range(warmup):
        plan.apply(xd, yd, precision=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.apply(xd, yd, precision=prec)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _stage_rooflines(plan, xd, yd, r, nnz, reps, workload=None):
    """Per precision: the stage table of one apply and the dominant stage's
    roofline."""
    from paper_2311_08595_amd import _lib as L
    bk, bm = plan.query(L.Q_BUCKET_K).tolist(), plan.query(L.Q_BUCKET_M).tolist()
    bl = plan.query(L.Q_BUCKET_LANES).tolist()
    bs = plan.query(L.Q_BUCKET_STACK).tolist()
    out = {}
    for prec in ("fp64", "fp32"):
        stages = stage_table(plan, xd, yd, prec, reps)
        prev = nnz
        for st_ in stages:
            if st_["kind"] == 2:
                st_["in_len"] = prev
                prev = st_["count"]
        work = stage_work(stages, bk, bm, r, bl, prec, bs)
        best, roof = roofline_of(stages, work, prec, r, workload)
        roof["avg_kernel_ms"] = best["ms"]
        roof["stages_ms_sum"] = sum(s_["ms"] for s_ in stages)
        out[prec] = dict(roofline=roof, stages_ms=[(s_["kind"], s_["size"], s_["count"], round(s_["ms"], 5))
                                                   for s_ in stages])
    return out


def bench_small(a):
    """The small uniform workload (n = 1000, m = 5000, sizes uniform on
    {2..5}, r = 5, x uniform on (0,1]): microseconds per STTSV (FP64 and FP32
    series), per captured NQZ iteration (20 shifted iterations, alpha = 1, one
    captured graph), and to 1e-8; the FP64 oracle beside it (one process: the
    whole graph is small)."""
    import torch
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import workloads as wl
    from oracle import nqz_ref, sttsv_ref
    w = wl.small_uniform(seed=1)
    n, r, m = w["n"], w["r"], len(w["eptr"]) - 1
    res = {"workload": w["name"], "n": n, "m": m, "nnz": int(len(w["eidx"])), "r": r}
    with st.Plan(w["eptr"], w["eidx"], n, r) as p:
        xd = torch.tensor(w["x"], dtype=torch.float64, device="cuda")
        yd = torch.empty_like(xd)
        for prec in ("fp64", "fp32"):
            dt = _timed_applies(p, xd, yd, prec, 200, 2000)
            res["sttsv_%s_us" % prec] = dt * 1e6
            res["sttsv_%s_hyperedges_per_s" % prec] = m / dt
        res.update(_stage_rooflines(p, xd, yd, r, len(w["eidx"]), 20))
        res["bound"] = ("launch/latency: %.1e series FMAs and %.2f MB per STTSV are well under a microsecond of "
                        "the chip at any roofline" % (sum(edge_fma(int(k), r) for k in np.diff(w["eptr"])),
                                                      20.0 * len(w["eidx"]) / 1e6))
        for use_graph in (True, False):
            p.solve(tol=1e-300, max_iter=20, shift=1.0, check_every=20, use_graph=use_graph, raise_on_notconv=False)
            torch.cuda.synchronize()
            reps = 20
            t0 = time.perf_counter()
            for _ in range(reps):
                _, info = p.solve(tol=1e-300, max_iter=20, shift=1.0, check_every=20, use_graph=use_graph,
                                  raise_on_notconv=False)
            dt = (time.perf_counter() - t0) / reps
            key = "shifted20_%s" % ("captured" if use_graph else "uncaptured")
            res[key] = {"seconds": dt, "us_per_iteration": dt * 1e6 / 20, "iterations": info["iterations"]}
        p.solve(tol=1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = p.solve(tol=1e-8)
        res["solve_1e8_fp64"] = {"seconds": time.perf_counter() - t0, "iterations": info["iterations"]}
    # the oracle on the host: one STTSV, 20 shifted iterations, and the solve to 1e-8
    t0 = time.perf_counter()
    sttsv_ref.sttsv(w["eptr"], w["eidx"], n, r, w["x"])
    t_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    nqz_ref.nqz(w["eptr"], w["eidx"], n, r, tol=0.0, max_iter=20, alpha=1.0)
    t_20 = time.perf_counter() - t0
    t0 = time.perf_counter()
    o = nqz_ref.nqz(w["eptr"], w["eidx"], n, r, tol=1e-8, max_iter=500)
    t_c = time.perf_counter() - t0
    res["oracle"] = {"cores": 1, "cpu": host_cpu(), "sttsv_us": t_s * 1e6, "shifted20_seconds": t_20,
                     "solve_1e8_seconds": t_c, "solve_1e8_iterations": o["iterations"]}
    log("[bench]   small uniform: FP64 STTSV %.1f us, captured iteration %.1f us, solve to 1e-8 %.2f ms "
        "(oracle %.1f ms / %.2f s)" % (res["sttsv_fp64_us"], res["shifted20_captured"]["us_per_iteration"],
                                       res["solve_1e8_fp64"]["seconds"] * 1e3, t_s * 1e3, t_c))
    return res


def bench_heavy(a):
    """The heavy-tail workload (n = 2e5, m = 2e6, sizes: w.p. 0.99 truncated
    geometric p = 0.4 on [2, 8], w.p. 0.01 uniform on [9, 50], r = 50, uniform
    membership): STTSV per precision with its dominant stage's roofline, and
    the solve to 1e-8 on the largest component (FP64, and FP32 series then
    FP64)."""
    import torch
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import workloads as wl
    w = wl.heavy_tail()
    n, r, m = w["n"], w["r"], len(w["eptr"]) - 1
    res = {"workload": w["name"], "n": n, "m": m, "nnz": int(len(w["eidx"])), "r": r}
    t0 = time.perf_counter()
    with st.Plan(w["eptr"], w["eidx"], n, r) as p:
        res["plan_s"] = time.perf_counter() - t0
        xd = torch.tensor(w["x"], dtype=torch.float64, device="cuda")
        yd = torch.empty_like(xd)
        for prec in ("fp64", "fp32"):
            res["untuned_%s_ms" % prec] = _timed_applies(p, xd, yd, prec, 20, 100) * 1e3
        if not a.no_tune:
            t0 = time.perf_counter()
            p.autotune(xd, reps=5)
            res["autotune_s"] = time.perf_counter() - t0
        y64 = None
        for prec in ("fp64", "fp32"):
            dt = _timed_applies(p, xd, yd, prec, 20, 100)
            res["sttsv_%s_ms" % prec] = dt * 1e3
            res["sttsv_%s_hyperedges_per_s" % prec] = m / dt
            if prec == "fp64":
                y64 = yd.clone()
        nz = y64 != 0
        res["fp32_max_rel_err_vs_fp64"] = float(((yd[nz] - y64[nz]).abs() / y64[nz].abs()).max())
        res.update(_stage_rooflines(p, xd, yd, r, len(w["eidx"]), 5, "heavy"))
    log("[bench]   heavy tail: FP64 %.3f ms, FP32 %.3f ms per STTSV" % (res["sttsv_fp64_ms"], res["sttsv_fp32_ms"]))
    e2, i2, n2, _ = wl.largest_component(w["eptr"], w["eidx"], n)
    solve = {"n_lcc": n2, "m_lcc": len(e2) - 1, "tol": 1e-8}
    with st.Plan(e2, i2, n2, r) as p2:
        if not a.no_tune:
            p2.autotune(torch.full((n2,), 1.0 / n2, dtype=torch.float64, device="cuda"), reps=5)
        for sched in ("fp64", "fp32_fp64"):
            p2.solve(tol=1e-8, schedule=sched)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = p2.solve(tol=1e-8, schedule=sched)
            solve[sched] = {"seconds": time.perf_counter() - t0, "iterations": info["iterations"],
                            "iters_fp32": info["iters_fp32"], "iters_fp64": info["iters_fp64"],
                            "criterion": info["criterion"]}
            log("[bench]   heavy tail solve %s: %.4f s, %d iterations" % (sched, solve[sched]["seconds"],
                                                                         info["iterations"]))
    res["solve"] = solve
    return res


def profile_apply(a):
    """Short run for a profiler: the plan autotuned as the headline run does
    it (unless --no-tune), then a plain device copy that marks the end of
    set-up (and, of known size, calibrates FETCH_SIZE / WRITE_SIZE), a few
    applies of each precision, and the stage-timed passes whose HIP-event
    times the profiler's averages are checked against."""
    import torch
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import _lib as L
    from paper_2311_08595_amd import workloads as wl
    w = {"zipf": lambda: wl.zipf_powerlaw(n=a.n, m=a.m), "heavy": wl.heavy_tail,
         "small": wl.small_uniform}[a.profile]()
    with st.Plan(w["eptr"], w["eidx"], w["n"], w["r"]) as p:
        xd = torch.tensor(w["x"], dtype=torch.float64, device="cuda")
        yd = torch.empty_like(xd)
        if not a.no_tune:
            # --tune-cache: later profiler passes reuse the first pass's
            # kernel choices (counter collection slows launches unevenly)
            p.autotune(xd, reps=5, cache_path=a.tune_cache)
        mib = a.calib_copy_mib or 256
        src = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[profile] %s: set-up done, %d MiB marker copy" % (w["name"], mib))
        bk, bm, bl = p.query(L.Q_BUCKET_K), p.query(L.Q_BUCKET_M), p.query(L.Q_BUCKET_LANES)
        bs = p.query(L.Q_BUCKET_STACK)
        for prec in ("fp64", "fp32"):
            for _ in range(a.steps):
                p.apply(xd, yd, precision=prec)
            torch.cuda.synchronize()
            stages = stage_table(p, xd, yd, prec, a.stage_reps)
            prev = len(w["eidx"])
            for st_ in stages:
                if st_["kind"] == 2:
                    st_["in_len"] = prev
                    prev = st_["count"]
            work = stage_work(stages, bk, bm, w["r"], bl, prec, bs)
            i = max(range(len(stages)), key=lambda j: stages[j]["ms"])
            kname, grid = stage_kernel(stages[i], prec, w["r"], work[i][3])
            log("[profile] %s %s: %d applies, %d stage-timed passes; dominant stage %s (kernel %s, grid %s): "
                "%.2f us by HIP events, %.4g FLOP, %.4g B algorithmic"
                % (w["name"], prec, a.steps, a.stage_reps, work[i][2], kname, grid, stages[i]["ms"] * 1e3,
                   work[i][0], work[i][1]))


def bench_batch(a):
    """256 hypergraphs (n log-uniform in [1e3, 1e5], m = 5n, r uniform in
    {3..12}, P(k) ~ k^-2.5 on [2, r], uniform membership), each restricted to
    its largest component, in one plan: batched STTSV throughput before and
    after autotuning, batched solve to 1e-8, and the sum of the per-graph
    solves for comparison."""
    import torch
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import workloads as wl
    log("[bench] batched workload: %d graphs" % a.batch_graphs)
    gs = []
    for g in range(a.batch_graphs):
        w = wl.batch_graph(g)
        e2, i2, n2, _ = wl.largest_component(w["eptr"], w["eidx"], w["n"])
        gs.append((e2, i2, n2, w["r"]))
    ntot = sum(g[2] for g in gs)
    mtot = sum(len(g[0]) - 1 for g in gs)
    t0 = time.perf_counter()
    pb = st.Plan.batch(gs)
    plan_s = time.perf_counter() - t0
    xd = torch.ones(ntot, dtype=torch.float64, device="cuda")
    yd = torch.empty_like(xd)
    res = {"graphs": len(gs), "n_total": ntot, "m_total": mtot, "plan_s": plan_s}

    def rate(prec):
        for _ in range(a.warmup):
            pb.apply(xd, yd, precision=prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(a.steps):
            pb.apply(xd, yd, precision=prec)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / a.steps
    for prec in ("fp64", "fp32"):
        dt = rate(prec)
        res["sttsv_%s" % prec] = {"ms": dt * 1e3, "hyperedges_per_s": mtot / dt}
    t0 = time.perf_counter()
    res["autotune_decisions"] = pb.autotune(xd, reps=3)
    res["autotune_s"] = time.perf_counter() - t0
    for prec in ("fp64", "fp32"):
        dt = rate(prec)
        res["sttsv_%s_tuned" % prec] = {"ms": dt * 1e3, "hyperedges_per_s": mtot / dt}
    for sched in ("fp64", "fp32_fp64"):
        pb.solve_batch(tol=1e-8, schedule=sched)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infos = pb.solve_batch(tol=1e-8, schedule=sched)
        dt = time.perf_counter() - t0
        its = [i["iterations"] for i in infos]
        res["solve_batch_%s" % sched] = {"seconds": dt, "iters_min": min(its), "iters_max": max(its),
                                         "all_converged": all(i["converged"] for i in infos)}
        log("[bench]   batched solve %s: %.4f s (iterations %d..%d)" % (sched, dt, min(its), max(its)))
    from paper_2311_08595_amd.warmstart import MpnnGraph, WarmStartNet, DEFAULT_WEIGHTS
    if os.path.exists(DEFAULT_WEIGHTS):
        net = WarmStartNet.load(DEFAULT_WEIGHTS)
        mgs = [MpnnGraph(e2, i2, n2, r2) for (e2, i2, n2, r2) in gs]
        x0 = torch.empty(ntot, dtype=torch.float64, device="cuda")

        def infer():
            off = 0
            for mg in mgs:
                net.warm_start(mg, out=x0[off:off + mg.n])
                off += mg.n
        infer()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infer()
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        res["net_inference_s"] = t_inf
        for sched in ("fp64", "fp32_fp64"):
            pb.solve_batch(tol=1e-8, schedule=sched, x0=x0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infos = pb.solve_batch(tol=1e-8, schedule=sched, x0=x0)
            dt = time.perf_counter() - t0
            its = [i["iterations"] for i in infos]
            res["solve_batch_net_start_%s" % sched] = {"seconds": dt + t_inf, "solve_seconds": dt,
                                                       "iters_min": min(its), "iters_max": max(its),
                                                       "all_converged": all(i["converged"] for i in infos)}
            log("[bench]   batched solve %s (learned start): %.4f s incl. %.4f s inference (iterations %d..%d)"
                % (sched, dt + t_inf, t_inf, min(its), max(its)))
    pb.close()
    tot = 0.0
    for (e2, i2, n2, r2) in gs:
        with st.Plan(e2, i2, n2, r2) as p1:
            p1.solve(tol=1e-8)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p1.solve(tol=1e-8)
            tot += time.perf_counter() - t0
    res["solve_single_sum_fp64_s"] = tot
    log("[bench]   sum of %d single-graph solves: %.4f s" % (len(gs), tot))
    return res


def coo_bytes(sizes, r):
    """COO storage (4-byte indices, 8-byte values) of the hypergraph's
    tensor: of its IOU non-zeros (one sorted index tuple per edge, Sec. III)
    and of every non-zero of the order-r blowup tensor (|beta(e)| = |e|!
    S(r,|e|) tuples of r indices per edge, Sec. II), the latter as log10."""
    from math import factorial, log10
    s2 = [[0] * (r + 1) for _ in range(r + 1)]
    s2[0][0] = 1
    for a_ in range(1, r + 1):
        for b_ in range(1, a_ + 1):
            s2[a_][b_] = b_ * s2[a_ - 1][b_] + s2[a_ - 1][b_ - 1]
    ks, cnt = np.unique(sizes, return_counts=True)
    iou = int(np.sum(cnt * (4 * ks + 8)))
    blow = sum(int(c) * factorial(int(k)) * s2[r][int(k)] for k, c in zip(ks, cnt)) * (4 * r + 8)
    return iou, log10(blow)


def bench_ccss(plan, w, xd, yd, reps):
    """Alg. 4 over the CCSS forest (Sec. III-IV) on the same plan: forest
    sizes, storage against COO, construction time, FP64 STTSV time against
    the leave-one-out kernels, and the largest relative difference."""
    import torch
    info = plan.ccss_build()
    sizes = np.diff(w["eptr"])
    iou, blow_log10 = coo_bytes(sizes, w["r"])
    ccss_bytes = 8 * info["nodes"] + 4 * info["leaves"]
    t_c = _timed_ccss(plan, xd, yd, reps)
    y_c = yd.clone()
    t_m = _timed_applies(plan, xd, yd, "fp64", 5, reps)
    nz = yd != 0
    naive_conv = int(np.sum(sizes * (sizes - 1)))
    return dict(levels=info["levels"], nodes=info["nodes"], roots=info["roots"],
                convolutions=info["convolutions"], leaves=info["leaves"],
                convolutions_naive=naive_conv, convolutions_no_sharing=int(np.sum((sizes - 1) * (sizes + 2) // 2 - 2 * (sizes >= 2))),
                build_ms=info["build_ms"], ccss_bytes=ccss_bytes, coo_iou_bytes=iou, coo_blowup_bytes_log10=blow_log10,
                coo_iou_over_ccss=iou / ccss_bytes, coo_blowup_over_ccss_log10=blow_log10 - math.log10(ccss_bytes),
                alg4_ms=t_c * 1e3, leave_one_out_ms=t_m * 1e3, alg4_over_leave_one_out=t_c / t_m,
                max_rel_diff=float(((y_c[nz] - yd[nz]).abs() / yd[nz].abs()).max()),
                workspace_device_bytes=info["device_bytes"])


def _timed_ccss(plan, xd, yd, reps):
    import torch
    for _ in range(3):
        plan.apply_ccss(xd, yd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.apply_ccss(xd, yd)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def bench_paper_synthetic(a):
    """The paper's synthetic sets S1-S4 (n=2500, m=25000, sizes 5, 10, ...,
    N_k for N_k = 30, 40, 50, 60, r = N_k): FP64 STTSV by the memoised
    kernels (plan as built, then autotuned once like the headline plan)
    against the NAIVE algorithm (Alg. 3) on the same GPU and plan, the
    shape of the paper's memoised-vs-naive comparison.  Work counts:
    truncated products per edge k(k-1) (naive, Sec. IV) vs 2(k-3) windowed
    ones (memoised); naive series FMAs k(k-1) r(r-1)/2 per edge."""
    import torch
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import workloads as wl
    rows = []
    reps = max(5, min(a.steps, 20))
    for nk in (30, 40, 50, 60):
        d = wl.paper_synthetic(nk)
        n, r = d["n"], d["r"]
        sizes = np.diff(d["eptr"])
        m = len(sizes)
        with st.Plan(d["eptr"], d["eidx"], n, r) as p:
            xd = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
            yd = torch.empty_like(xd)

            def run(f):
                for _ in range(3):
                    f(xd, yd)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    f(xd, yd)
                torch.cuda.synchronize()
                return (time.perf_counter() - t0) / reps
            t_built = run(lambda x, y: p.apply(x, y, precision="fp64"))
            t_naive = run(p.apply_naive)
            cc = bench_ccss(p, d, xd, yd, reps)
            if not a.no_tune:   # the same one-off tuning as the headline plan
                p.autotune(xd, reps=5)
                t_memo = run(lambda x, y: p.apply(x, y, precision="fp64"))
            else:
                t_memo = t_built
        k = sizes.astype(np.float64)
        naive_fma = float(np.sum(k * (k - 1)) * r * (r - 1) / 2)
        memo_fma = float(sum(edge_fma(int(kk), r) * int(c) for kk, c in zip(*np.unique(sizes, return_counts=True))))
        row = {"set": "S%d" % (nk // 10 - 2), "r": r, "m": m, "nnz": int(len(d["eidx"])),
               "memoised_ms": t_memo * 1e3, "memoised_as_built_ms": t_built * 1e3,
               "naive_ms": t_naive * 1e3, "speedup": t_naive / t_memo,
               "memoised_hyperedges_per_s": m / t_memo, "naive_hyperedges_per_s": m / t_naive,
               "products_naive": int(np.sum(sizes * (sizes - 1))),
               "products_memoised": int(np.sum(np.where(sizes >= 4, 2 * (sizes - 3), (sizes == 3).astype(np.int64)))),
               "naive_tflops": 2 * naive_fma / t_naive / 1e12, "memoised_tflops": 2 * memo_fma / t_memo / 1e12,
               "ccss": cc}
        rows.append(row)
        log("[bench]   %s (r=%d): memoised %.3f ms (as built %.3f), naive %.3f ms (%.1fx), naive %.1f TFLOP/s, "
            "Alg. 4 over CCSS %.3f ms (%d nodes)"
            % (row["set"], r, row["memoised_ms"], row["memoised_as_built_ms"], row["naive_ms"], row["speedup"],
               row["naive_tflops"], cc["alg4_ms"], cc["nodes"]))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--m", type=int, default=5_000_000)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-edges", type=int, default=2000000)
    ap.add_argument("--stage-reps", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-synthetic", action="store_true", help="skip the S1-S4 memoised-vs-naive comparison")
    ap.add_argument("--synthetic-only", action="store_true",
                    help="run only the S1-S4 memoised-vs-naive comparison (prints its rows as JSON)")
    ap.add_argument("--no-tune", action="store_true", help="time the plan as built, without autotuning")
    ap.add_argument("--batch-graphs", type=int, default=256)
    ap.add_argument("--no-small", action="store_true", help="skip the small uniform workload (n=1e3, r=5)")
    ap.add_argument("--no-ccss", action="store_true", help="skip the CCSS forest / Alg. 4 comparison")
    ap.add_argument("--no-heavy", action="store_true", help="skip the heavy-tail workload (n=2e5, r=50)")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle worker processes (0: the host's share, <= 16)")
    ap.add_argument("--profile", choices=["zipf", "heavy", "small"], default=None,
                    help="only run --steps applies of each precision on one workload (for counter runs)")
    ap.add_argument("--tune-cache", default=None, help="autotuner choice file (read, then appended to)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the STTSV path is built and measured on a single "
              "MI355X (multi-GPU sharding is a design note, not part of this build).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import workloads as wl

    if a.profile:
        torch.cuda.set_device(0)
        profile_apply(a)
        return
    if a.synthetic_only:
        torch.cuda.set_device(0)
        log("[bench] paper synthetic sets S1-S4: memoised vs naive (Alg. 3)")
        print(json.dumps({"paper_synthetic": bench_paper_synthetic(a)}), flush=True)
        return
    log("[bench] generating workload")
    w = wl.zipf_powerlaw(n=a.n, m=a.m)
    n, r, m = w["n"], w["r"], len(w["eptr"]) - 1
    cpu = None
    if not a.no_cpu:
        # the oracle's worker processes are forked before this process touches the GPU
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(w, a.cpu_edges, a.cpu_procs or oracle_procs())
        log("[bench]   %.3e hyperedges/s on %d processes" % (cpu["value"], cpu["cores"]))
    torch.cuda.set_device(0)
    log("[bench] planning n=%d m=%d nnz=%d r=%d" % (n, m, len(w["eidx"]), r))
    t0 = time.perf_counter()
    plan = st.Plan(w["eptr"], w["eidx"], n, r)
    plan_s = time.perf_counter() - t0
    xd = torch.tensor(w["x"], dtype=torch.float64, device="cuda")
    yd = torch.empty_like(xd)

    if a.calib_copy_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings
        # calibrate the counters taken on the STTSV kernels of the same run
        src = torch.ones(a.calib_copy_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy of %d MiB done" % a.calib_copy_mib)
        del src, dst

    from paper_2311_08595_amd import _lib as L

    def time_apply(prec):
        for _ in range(a.warmup):
            plan.apply(xd, yd, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            plan.apply(xd, yd, precision=prec)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / a.steps

    # the plan as built, then autotuned once (kernel variants and stream
    # lanes; both are setup like the plan itself and never change a bit of y)
    untuned = {}
    for prec in ("fp64", "fp32"):
        log("[bench] timing STTSV %s (plan as built)" % prec)
        untuned[prec] = time_apply(prec)
    tune_s = None
    if not a.no_tune:
        t0 = time.perf_counter()
        plan.autotune(xd, reps=5)
        tune_s = time.perf_counter() - t0
        log("[bench] autotuned in %.2f s" % tune_s)
    res = {"bucket_k": plan.query(L.Q_BUCKET_K).tolist(), "bucket_m": plan.query(L.Q_BUCKET_M).tolist(),
           "bucket_l": plan.query(L.Q_BUCKET_LANES).tolist(), "bucket_s": plan.query(L.Q_BUCKET_STACK).tolist()}
    for prec in ("fp64", "fp32"):
        log("[bench] timing STTSV %s" % prec)
        dt = time_apply(prec) if tune_s is not None else untuned[prec]
        stages = stage_table(plan, xd, yd, prec, a.stage_reps)
        # terms read by each reduction level: nnz at level 0, at most the previous
        # level's chunk count above it
        prev = len(w["eidx"])
        for st_ in stages:
            if st_["kind"] == 2:
                st_["in_len"] = prev
                prev = st_["count"]
        res[prec] = dict(ms=dt * 1e3, stages=stages, y=yd.clone())
        log("[bench]   %s: %.3f ms/STTSV, %.3e hyperedges/s" % (prec, dt * 1e3, m / dt))
    # error of the FP32-series result against the FP64 path (which the tests
    # hold to 1e-12 of the oracle), over vertices with y != 0
    y64, y32 = res["fp64"].pop("y"), res["fp32"].pop("y")
    nz = y64 != 0
    fp32_err = float(((y32[nz] - y64[nz]).abs() / y64[nz].abs()).max())

    out = {
        "metric": "STTSV hyperedges/s",
        "value": m / (res["fp64"]["ms"] * 1e-3),
        "unit": "hyperedges/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res["fp64"]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "n": n, "m": m, "nnz": int(len(w["eidx"])), "r": r,
                   "sizes": "P(k)~k^-2.5 on [2,25]", "membership": "Zipf(1.0)",
                   "parallelism": "1 GPU",
                   "plan": "autotuned once before timing (kernel variants, stream lanes; bitwise-identical y)"
                   if tune_s is not None else "as built"},
        "untuned_ms_per_step": {"fp64": untuned["fp64"] * 1e3, "fp32": untuned["fp32"] * 1e3},
        "autotune_s": tune_s,
    }
    from paper_2311_08595_amd import _lib
    bk, bm = res["bucket_k"], res["bucket_m"]
    for prec in ("fp64", "fp32"):
        res[prec]["work"] = stage_work(res[prec]["stages"], bk, bm, r, res["bucket_l"], prec, res["bucket_s"])
    best, roof = roofline_of(res["fp64"]["stages"], res["fp64"]["work"], "fp64", r, "zipf")
    roof["avg_kernel_ms"] = best["ms"]
    out["roofline"] = roof
    best32, roof32 = roofline_of(res["fp32"]["stages"], res["fp32"]["work"], "fp32", r, "zipf")
    roof32["avg_kernel_ms"] = best32["ms"]
    out["fp32_series"] = {"value": m / (res["fp32"]["ms"] * 1e-3), "ms_per_step": res["fp32"]["ms"],
                          "max_rel_err_vs_fp64": fp32_err, "roofline": roof32}
    out["stages_fp64_ms"] = [(s["kind"], s["size"], s["count"], round(s["ms"], 5)) for s in res["fp64"]["stages"]]
    out["stages_fp32_ms"] = [(s["kind"], s["size"], s["count"], round(s["ms"], 5)) for s in res["fp32"]["stages"]]
    out["plan_s"] = plan_s
    if not a.no_ccss:
        log("[bench] CCSS forest and Alg. 4")
        try:   # a failure here must not cost the headline line
            out["ccss"] = bench_ccss(plan, w, xd, yd, 20)
            log("[bench]   %d nodes, built in %.1f ms; Alg. 4 %.3f ms vs %.3f ms; COO(IOU)/CCSS %.2f"
                % (out["ccss"]["nodes"], out["ccss"]["build_ms"], out["ccss"]["alg4_ms"],
                   out["ccss"]["leave_one_out_ms"], out["ccss"]["coo_iou_over_ccss"]))
        except Exception as exc:
            out["ccss"] = {"error": str(exc)}
            log("[bench]   CCSS failed: %s" % exc)
    plan.close()

    # prefix reuse (FP64, sizes 4..7): a plan with the flag; per-bucket share
    # of edges that take the shared product phi_0 phi_1 from their run, the
    # series FMAs that saves, and the time it takes
    log("[bench] prefix reuse")
    with st.Plan(w["eptr"], w["eidx"], n, r, flags=L.FLAG_PREFIX_REUSE) as pr:
        runs = pr.query(L.Q_BUCKET_RUNS)
        for _ in range(a.warmup):
            pr.apply(xd, yd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            pr.apply(xd, yd)
        torch.cuda.synchronize()
        dt_r = (time.perf_counter() - t0) / a.steps
    total_fma = sum(edge_fma(k, r) * m for k, m in zip(bk, bm))
    rows, share, saved = [], 0, 0.0
    for k, m, nr in zip(bk, bm, runs.tolist()):
        if nr > 0:
            W = r - k + 1
            rows.append({"k": k, "edges": m, "runs": nr, "edges_sharing": m - nr})
            share += m - nr
            saved += (m - nr) * W * (W - 1) / 2
    reuse_m = sum(x["edges"] for x in rows)
    out["prefix_reuse"] = {"buckets": rows, "share_fraction": share / max(reuse_m, 1),
                           "fma_saved_fraction_of_all_edges": saved / total_fma,
                           "ms_per_step": dt_r * 1e3, "time_vs_plain": dt_r / (res["fp64"]["ms"] * 1e-3)}
    log("[bench]   reuse: %.1f%% of size-4..7 edges share, %.1f%% of series FMAs saved, %.3f ms (plain %.3f ms)"
        % (100 * share / max(reuse_m, 1), 100 * saved / total_fma, dt_r * 1e3, res["fp64"]["ms"]))

    if not a.no_solve:
        log("[bench] largest component + solves")
        e2, i2, n2, _ = wl.largest_component(w["eptr"], w["eidx"], n)
        solve = {"n_lcc": n2, "m_lcc": len(e2) - 1, "tol": 1e-8}
        with st.Plan(e2, i2, n2, r) as p2:
            if not a.no_tune:   # the same one-off tuning as the headline plan
                t0 = time.perf_counter()
                p2.autotune(torch.full((n2,), 1.0 / n2, dtype=torch.float64, device="cuda"), reps=5)
                solve["autotune_s"] = time.perf_counter() - t0

            def timed(sched, x0=None, pre=0.0):
                p2.solve(tol=1e-8, schedule=sched, x0=x0)   # warm-up (graph capture)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xs, info = p2.solve(tol=1e-8, schedule=sched, x0=x0)
                dt = time.perf_counter() - t0
                out_x[(sched, x0 is None)] = xs
                return dict(seconds=dt + pre, solve_seconds=dt, iterations=info["iterations"],
                            iters_fp32=info["iters_fp32"], iters_fp64=info["iters_fp64"],
                            lambda_max=info["lambda_max"], criterion=info["criterion"])
            out_x = {}
            for sched in ("fp64", "fp32_fp64"):
                solve[sched] = timed(sched)
                log("[bench]   solve %s (uniform start): %.4f s, %d iterations"
                    % (sched, solve[sched]["seconds"], solve[sched]["iterations"]))
            # the FP32->FP64 result against the FP64 one (same tolerance, same start)
            xa, xb = out_x[("fp64", True)], out_x[("fp32_fp64", True)]
            solve["fp32_fp64"]["max_rel_diff_vs_fp64"] = float(((xb - xa).abs() / xa).max())
            # control: degree start d^(1/(r-1)) (the first NQZ iterate from the uniform start)
            d = np.bincount(i2, minlength=n2).astype(np.float64)
            xdeg = torch.tensor(d ** (1.0 / (r - 1)), dtype=torch.float64, device="cuda")
            solve["degree_start_fp64"] = timed("fp64", xdeg)
            log("[bench]   solve fp64 (degree start): %.4f s, %d iterations"
                % (solve["degree_start_fp64"]["seconds"], solve["degree_start_fp64"]["iterations"]))
            # learned warm start (network trained on n=1e4 graphs), inference timed with the solve
            from paper_2311_08595_amd.warmstart import MpnnGraph, WarmStartNet, DEFAULT_WEIGHTS
            if os.path.exists(DEFAULT_WEIGHTS):
                net = WarmStartNet.load(DEFAULT_WEIGHTS)
                t0 = time.perf_counter()
                mg = MpnnGraph(e2, i2, n2, r)
                prep = time.perf_counter() - t0
                net.warm_start(mg)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x0 = net.warm_start(mg)
                torch.cuda.synchronize()
                infer = time.perf_counter() - t0
                solve["net_graph_prep_s"] = prep
                solve["net_inference_s"] = infer
                for sched in ("fp64", "fp32_fp64"):
                    solve["net_start_" + sched] = timed(sched, x0, pre=infer)
                    log("[bench]   solve %s (learned start): %.4f s incl. %.4f s inference, %d iterations"
                        % (sched, solve["net_start_" + sched]["seconds"], infer,
                           solve["net_start_" + sched]["iterations"]))
            try:   # a failure here must not cost the headline line
                # another STTSV consumer: Z-eigenpair by the shifted power method
                # (SS-HOPM), shift on the scale of B x^r at the unit start
                x1 = torch.ones(n2, dtype=torch.float64, device="cuda")
                x1 /= float(np.sqrt(n2))
                lam0, _ = p2.contract(x1)
                p2.zeig_sshopm(None, alpha=lam0, tol=1e-10, max_iter=300, raise_on_notconv=False)   # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, zi = p2.zeig_sshopm(None, alpha=lam0, tol=1e-10, max_iter=300, raise_on_notconv=False)
                dt = time.perf_counter() - t0
                solve["sshopm_fp64"] = dict(seconds=dt, iterations=zi["iterations"], converged=zi["converged"],
                                            lambda_=zi["lambda_"], residual=zi["residual"], alpha=lam0,
                                            ms_per_update=dt * 1e3 / max(zi["iterations"], 1))
                log("[bench]   SS-HOPM Z-eigenpair: %.4f s, %d updates (%.3f ms each), residual/lambda %.1e"
                    % (dt, zi["iterations"], dt * 1e3 / max(zi["iterations"], 1),
                       zi["residual"] / zi["lambda_"] if zi["lambda_"] else float("nan")))
                # cost of one update against one STTSV of the same plan: fixed
                # update counts (tol = 0), the difference over the extra updates
                def zt(k):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    p2.zeig_sshopm(None, alpha=lam0, tol=0.0, max_iter=k, raise_on_notconv=False)
                    return time.perf_counter() - t
                zt(8)
                t8, t40 = min(zt(8) for _ in range(3)), min(zt(40) for _ in range(3))
                y2 = torch.empty_like(x1)
                st_ms = _timed_applies(p2, x1, y2, "fp64", 5, 50) * 1e3
                solve["sshopm_fp64"].update(update_ms=(t40 - t8) * 1e3 / 32, sttsv_ms=st_ms)
                log("[bench]   SS-HOPM update %.3f ms against one FP64 STTSV %.3f ms"
                    % ((t40 - t8) * 1e3 / 32, st_ms))
            except Exception as exc:
                solve["sshopm_fp64"] = {"error": str(exc)}
                log("[bench]   SS-HOPM failed: %s" % exc)
            try:   # symmetric CP decomposition: one objective + gradient (R FP64 STTSVs) and a short descent
                R = 4
                gen = torch.Generator(device="cuda").manual_seed(7)
                A = torch.rand((R, n2), dtype=torch.float64, device="cuda", generator=gen)
                A /= A.norm(dim=1, keepdim=True)
                lam = torch.ones(R, dtype=torch.float64, device="cuda")
                p2.cp_objective_grad(A, lam)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(5):
                    f, _, _ = p2.cp_objective_grad(A, lam)
                eval_ms = (time.perf_counter() - t0) * 1e3 / 5
                t0 = time.perf_counter()
                ci = p2.cp_descent(A.clone(), lam.clone(), 10, 1.0)
                desc_s = time.perf_counter() - t0
                solve["sym_cp_r4"] = dict(eval_ms=eval_ms, sttsv_ms=solve.get("sshopm_fp64", {}).get("sttsv_ms"),
                                          descent_10_s=desc_s, f0=ci["f0"], f=ci["f"], norm2=ci["norm2"],
                                          halvings=ci["halvings"])
                log("[bench]   symmetric CP (R=4): %.3f ms per objective+gradient; 10 descent steps %.4f s, "
                    "f/||B||^2 %.4f -> %.4f" % (eval_ms, desc_s, ci["f0"] / ci["norm2"], ci["f"] / ci["norm2"]))
            except Exception as exc:
                solve["sym_cp_r4"] = {"error": str(exc)}
                log("[bench]   symmetric CP failed: %s" % exc)
        out["solve"] = solve
    if not a.no_batch:
        out["batched"] = bench_batch(a)
        # the warm-start target: warm-started batched FP32->FP64 solve (inference
        # included) against the plain FP64 solves of the same graphs one by one,
        # and, for the n=1e6 graph, the warm-started FP32->FP64 single solve
        # against its plain FP64 solve
        b = out["batched"]
        tgt = {}
        if "solve_batch_net_start_fp32_fp64" in b:
            # the network's gain at equal batching: warm-started batched FP32->FP64
            # (inference included) against the plain batched FP64 solve
            w_s = b["solve_batch_net_start_fp32_fp64"]["seconds"]
            tgt["batched_warm_fp32_fp64_s"] = w_s
            tgt["batched_plain_fp64_s"] = b["solve_batch_fp64"]["seconds"]
            tgt["batched_met"] = w_s < b["solve_batch_fp64"]["seconds"]
            # batching alone, for context: the same graphs solved one by one
            tgt["single_plain_fp64_sum_s"] = b["solve_single_sum_fp64_s"]
            tgt["batched_warm_vs_sequential_plain"] = w_s < b["solve_single_sum_fp64_s"]
        sv = out.get("solve", {})
        if "net_start_fp32_fp64" in sv:
            tgt["n1e6_warm_fp32_fp64_s"] = sv["net_start_fp32_fp64"]["seconds"]
            tgt["n1e6_plain_fp64_s"] = sv["fp64"]["seconds"]
            tgt["n1e6_met"] = sv["net_start_fp32_fp64"]["seconds"] < sv["fp64"]["seconds"]
        out["warm_start_target"] = tgt
    if not a.no_synthetic:
        log("[bench] paper synthetic sets S1-S4: memoised vs naive (Alg. 3)")
        out["paper_synthetic"] = bench_paper_synthetic(a)
    if not a.no_small:
        log("[bench] small uniform workload")
        out["small_uniform"] = bench_small(a)
    if not a.no_heavy:
        log("[bench] heavy-tail workload")
        out["heavy_tail"] = bench_heavy(a)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
