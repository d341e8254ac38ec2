#!/usr/bin/env python3
"""Throughput of the operator-split reaction-diffusion step on one MI355X.

Default workload (batched): 256 realizations of the A+B<->C system on the
40^3 x 6 Kuhn lattice (384,000 tets, 3 species) plus 64 realizations of its
20^3 x 6 variant (48,000 tets), advanced together by the batching engine
(hipGraph-captured chunks of periods).  A "step" is one period tau of every
realization.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload batched|plain]
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the device code's tokens: comments and layout do not count,
    so a measured traffic file stays valid across edits that change neither."""
    import re

    h = hashlib.sha256()
    for f in ("rdos_kernels.hip", "rdos_sampling.h", "rdos_internal.h"):
        with open(os.path.join(ROOT, "paper_1512_03126_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel, workload):
    """HBM bytes per launch of `kernel` measured by rocprofv3 counters for
    this workload, if the kernel sources have not changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_sources") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def scan_bytes(sims, models):
    """Bytes the occupancy-driven scan must move in the period that starts
    from the current state of every realization (the units and per-unit
    figures of the roofline):
      one map byte per four tets and species (read; the map is not cleared:
      its bytes carry the tag of the period they mark),
      16 B per flagged four-tet vector of one species (the count read),
      16 B per such vector again (its clear),
      4 + 4 S B per tet with molecules (its queue entry)."""
    import numpy as np

    total = 0
    for sim, m in zip(sims, models):
        T, S = m.n_tets, m.n_species
        Tp = (T + 3) // 4 * 4
        stride = ((Tp // 4) + 15) // 16 * 16
        for r in range(m.n_realizations):
            c = np.zeros((S, Tp), np.int32)
            c[:, :T] = sim.get_counts(None, realization=r)
            vec = (c != 0).reshape(S, Tp // 4, 4).any(axis=2)   # [S][groups]: flagged vectors
            tets = int((c != 0).any(axis=0).sum())
            total += S * stride + 32 * int(vec.sum()) + (4 + 4 * S) * tets
    return total


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor()


def oracle_baseline(model, periods):
    """The oracle as it stands, single thread, on one realization."""
    import oracle

    sim = oracle.OracleSim.from_model(model)
    t0 = time.perf_counter()
    sim.run_steps(periods)
    dt = time.perf_counter() - t0
    return periods * model.n_tets * model.n_species / dt, dt


def oracle_baseline_threads(model, periods, threads):
    """The oracle as it stands on `threads` host threads at once, one
    independent realization (its own seed) per thread, as the batched
    workload is independent realizations; the C oracle keeps no global state
    and ctypes releases the GIL during its calls."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    sims = [oracle.OracleSim.from_model(model, seed=1 + i) for i in range(threads)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda o: o.run_steps(periods), sims))
    dt = time.perf_counter() - t0
    return threads * periods * model.n_tets * model.n_species / dt, dt


def build_batched():
    import workloads as W

    big = W.abc_lattice(n=40, a=0.1e-6, seed=1, n_realizations=256)
    small = W.abc_lattice(n=20, a=0.1e-6, seed=2, n_realizations=64)
    return [big, small]


def make_sims(P, models):
    sims = []
    for m in models:
        s = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, n_realizations=m.n_realizations,
                         tau_scale=m.tau_scale)
        for r in range(m.n_realizations):
            for q in range(m.n_species):
                s.set_counts(q, m.init[r, q], realization=r)
        sims.append(s)
    return sims


def run_engine(P, e, sims, periods):
    """All simulations start from the same chunk (held while they are
    admitted), run `periods` periods, and are released."""
    P.rdos_engine_hold(e, True)
    tks = [P.rdos_engine_submit(e, s.h, periods, 1.0) for s in sims]
    P.rdos_engine_hold(e, False)
    P.rdos_engine_drain(e)
    for t in tks:
        P.rdos_engine_release(e, t)


def settle_engine(P, e, sims, max_rounds=8):
    """Untimed: runs the work until the engine's tuner has settled on a
    launch shape for it (each round is long enough for the tuner's whole
    candidate list), then one more chunk so that the graph of the chosen
    shape is captured before anything is timed.  Returns the periods run."""
    periods = 0
    for _ in range(max_rounds):
        if P.rdos_engine_launch_shape(e)["source"] != "default":
            break
        run_engine(P, e, sims, 192)
        periods += 192
    chunk = P.rdos_engine_launch_shape(e)["chunk"]
    run_engine(P, e, sims, 2 * chunk)
    return periods + 2 * chunk


def variant_models(name):
    """Models and method options of the widened rows, each timed like the
    batched mix: the same 256 + 64 realizations with another method option,
    a surface of the same size and occupancy, six and ten species."""
    import numpy as np

    import workloads as W

    if name in ("reference", "transfer_form_1", "first_order", "tau_outliers_10"):
        opts = {"transfer_form_1": {"transfer_form": 1}, "first_order": {"occupancy_correction": False},
                "tau_outliers_10": {"tau_outliers": 10}}.get(name, {})
        return build_batched(), opts
    if name == "six_species":
        # A+B<->C plus D -> E -> F -> D at 1/s, D, E, F as many as A, placed elsewhere
        out = []
        for m in build_batched():
            init = np.concatenate([m.init] + [np.roll(m.init[:, 0:1], 7919 * (q + 1), axis=2) for q in range(3)],
                                  axis=1)
            out.append(W.Model(m.name + "_six", m.xyz, m.tets, list(m.D) + [1e-12, 1e-12, 1e-12],
                               list(m.reactions) + [([3], [4], 1.0), ([4], [5], 1.0), ([5], [3], 1.0)],
                               np.ascontiguousarray(init), m.t_end, m.seed))
        return out, {}
    if name == "ten_species":
        # the chemistry of the 10-species stand-in for the model of Sec. III.C
        # (4 reversible pairs, D of 10-100 um^2/s) on the batched meshes, each
        # species as many molecules as A, placed elsewhere
        chem = W.ten_species(seed=1)
        out = []
        for m in build_batched():
            init = np.concatenate([np.roll(m.init[:, 0:1], 7919 * q, axis=2) for q in range(10)], axis=1)
            out.append(W.Model(m.name + "_ten", m.xyz, m.tets, list(chem.D), list(chem.reactions),
                               np.ascontiguousarray(init), m.t_end, m.seed))
        return out, {}
    if name == "surface":
        # 400 x 480 cells of 0.1 um, two triangles each (384,000), 3854 A and 3854 B
        # per realization placed uniformly (equal areas); surface A+B<->C with
        # about the pair and decay rates of the volume mix
        xyz, tris = W.triangle_lattice(400, 480, 0.1e-6)
        T = tris.shape[0]
        rng = np.random.default_rng(5)
        init = np.zeros((256, 3, T), np.int32)
        for r in range(256):
            for q in range(2):
                np.add.at(init[r, q], rng.integers(0, T, 3854), 1)
        area = 0.5 * (0.1e-6) ** 2
        k2 = 10.0 * W.N_A * area  # m^2/(mol s): 10 /s per pair in one triangle
        m = W.Model("surface_abc_384k", xyz, tris, [1e-12, 1e-12, 0.5e-12], [([0, 1], [2], k2), ([2], [0, 1], 10.0)],
                    init, 0.1, 1)
        return [m], {}
    raise ValueError(name)


def run_variants(P, args):
    """Throughput of the widened rows on the engine (the default launch-shape
    tuning, warm-up, then --steps timed periods each)."""
    res = {}
    for name in ("reference", "transfer_form_1", "first_order", "tau_outliers_10", "six_species", "ten_species",
                 "surface"):
        models, opts = variant_models(name)
        sims = []
        for m in models:
            sims.append(P.Simulation.from_model(m, **opts))
        upd = sum(m.n_realizations * m.n_tets * m.n_species for m in models)
        e = P.rdos_engine_create(0, 0)
        run_engine(P, e, sims, max(args.warmup, 1))
        settle_engine(P, e, sims)
        t0 = time.perf_counter()
        run_engine(P, e, sims, args.steps)
        dt = time.perf_counter() - t0
        shape = P.rdos_engine_launch_shape(e)
        P.rdos_engine_destroy(e)
        for x in sims:
            x.close()
        res[name] = {"updates_per_s": round(args.steps * upd / dt, 1), "ms_per_period": round(dt / args.steps * 1e3, 4),
                     "updates_per_period": upd, "species": models[0].n_species, "cells": [m.n_tets for m in models],
                     "realizations": [m.n_realizations for m in models], "launch_shape": shape}
        log(f"{name}: {res[name]['updates_per_s']:.3e} upd/s, {res[name]['ms_per_period']:.4f} ms/period")
    return res


def run_serving(P, args):
    """Poisson arrivals of independent requests (jittered lattices of 1e4-1e6
    tets, 1-6 species, random reactions), each asking for a fixed number of
    periods; admission by HBM budget, continuous batching on the device."""
    import numpy as np

    import workloads as W

    rng = np.random.default_rng(args.seed)
    arrivals = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / args.rate)
        if t > args.duration:
            break
        arrivals.append(t)
    log(f"serving: {len(arrivals)} requests over {args.duration:.0f} s (rate {args.rate}/s), "
        f"{args.request_steps} periods each, budget {args.budget_gb} GB")
    e = P.rdos_engine_create(0, int(args.budget_gb * (1 << 30)))
    pending = {}  # ticket -> (sim, scheduled arrival, updates)
    lat, total_updates, tets = [], 0.0, []
    parts, subm, submitted = [], [], {}
    t0 = time.perf_counter()
    last_done = t0

    def collect(block=False):
        nonlocal total_updates, last_done
        for tk in list(pending):
            done, _ = P.rdos_engine_poll(e, tk)
            if done:
                sim, sched, upd = pending.pop(tk)
                now = time.perf_counter()
                parts.append(P.rdos_engine_ticket_times(e, tk))
                subm.append(submitted.pop(tk) - (t0 + sched))
                P.rdos_engine_release(e, tk)
                sim.close()
                lat.append(now - (t0 + sched))
                total_updates += upd
                last_done = now

    # requests are generated ahead of their arrival by a small thread pool
    # (request i draws from its own seeded stream, so the mix is deterministic)
    from concurrent.futures import ThreadPoolExecutor

    pool = ThreadPoolExecutor(max_workers=6)
    window = {}

    def ahead(i):
        for j in range(i, min(i + 48, len(arrivals))):
            if j not in window:
                window[j] = pool.submit(W.serving_request, np.random.default_rng([args.seed, j]))

    for i, sched in enumerate(arrivals):
        ahead(i)
        m = window.pop(i).result()
        while time.perf_counter() - t0 < sched:
            collect()
            time.sleep(0.0005)
        sim = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, tau_scale=None)
        for q in range(m.n_species):
            sim.set_counts(q, m.init[0, q])
        tk = P.rdos_engine_submit(e, sim.h, args.request_steps, 1.0)
        submitted[tk] = time.perf_counter()
        pending[tk] = (sim, sched, float(args.request_steps) * m.n_tets * m.n_species)
        tets.append(m.n_tets)
        if (i + 1) % 200 == 0:
            log(f"  submitted {i + 1}, done {len(lat)}, in flight {len(pending)}")
    last_log = time.perf_counter()
    while pending:
        collect()
        time.sleep(0.0005)
        if time.perf_counter() - last_log > 5.0:
            last_log = time.perf_counter()
            log(f"  draining: done {len(lat)}, in flight {len(pending)}")
    pool.shutdown()
    wall = last_done - t0
    st = P.rdos_engine_stats(e)
    P.rdos_engine_destroy(e)
    lat_ms = np.sort(np.array(lat) * 1e3)
    br = {"host_before_submit": np.array(subm) * 1e3}
    for k in ("wait_s", "setup_s", "join_s", "run_s"):
        br[k.replace("_s", "")] = np.array([p_[k] for p_ in parts]) * 1e3
    breakdown = {k: {"p50_ms": round(float(np.percentile(v, 50)), 3), "p99_ms": round(float(np.percentile(v, 99)), 3)}
                 for k, v in br.items()}
    res = {"value": total_updates / wall, "wall_s": wall, "requests": len(lat),
           "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
           "latency_parts": breakdown,
           "mean_tets": float(np.mean(tets)), "device_busy_s": st["busy_s"],
           "device_updates_per_busy_s": st["updates"] / max(st["busy_s"], 1e-9)}
    log(f"serving: {res['value']:.3e} upd/s aggregate, p50 {res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms, "
        f"{res['requests']} requests, mean {res['mean_tets']:.0f} tets")
    log("serving latency parts (p50 / p99 ms): " + ", ".join(f"{k} {v['p50_ms']:.2f} / {v['p99_ms']:.2f}"
                                                             for k, v in breakdown.items()))
    return res


def timing_pass_ids(ids, name_of, first_copy, launches, where):
    """The dispatches of the timing pass in a profiled run of this script:
    the last 2 x `launches` step-kernel dispatches before the bandwidth
    probe's first copy, which must alternate scan_kernel, update_kernel (one
    pair per period; anything else, such as a fused or two-chain shape, is
    refused).  Returns {kernel: [ids]}."""
    steps = [d for d in ids if d < first_copy and ("scan_kernel" in name_of(d) or "update_kernel" in name_of(d))]
    last = steps[-2 * launches:]
    want = ["scan_kernel", "update_kernel"] * launches
    if len(last) != 2 * launches or any(k not in name_of(d) for k, d in zip(want, last)):
        raise SystemExit(f"{where}: the last {2 * launches} step-kernel dispatches before the copy probe are not "
                         f"{launches} scan/update pairs (was the launch shape fixed to a two-launch one?)")
    return {"scan_kernel": last[0::2], "update_kernel": last[1::2]}


def write_traffic(fetch_csv, write_csv, launches, command, out_dir=None):
    """Turns two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE) into profiles/<kernel>_batched_traffic.json for both step
    kernels: the mean over the last `launches` dispatches of each kernel (the
    timing pass, launched directly), in bytes, each counter scaled so that the
    1 GiB copy of the bandwidth probe in the same run reads 1 GiB and writes
    1 GiB."""
    import collections
    import csv

    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        disp = collections.defaultdict(float)
        name = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                d = int(r["Dispatch_Id"])
                disp[d] += float(r["Counter_Value"])
                name[d] = r["Kernel_Name"]
        copies = sorted(d for d in disp if "bandwidth_copy_kernel" in name[d])
        if not copies:
            raise SystemExit(f"no bandwidth_copy_kernel dispatch in {path}")
        pass_ids = timing_pass_ids(sorted(disp), lambda d: name[d], copies[0], launches, path)

        def mean_kib(k, n):
            ds = pass_ids[k] if k in pass_ids else copies[-n:]
            return sum(disp[d] for d in ds) / len(ds), len(ds)
        copy_kib, _ = mean_kib("bandwidth_copy_kernel", 5)
        scale = (1 << 30) / 1024 / copy_kib
        per[counter] = {k: mean_kib(k, launches) for k in ("scan_kernel", "update_kernel")}
        per[counter]["scale"] = scale
        per[counter]["copy_kib"] = copy_kib
    for k in ("scan_kernel", "update_kernel"):
        fb = per["FETCH_SIZE"][k][0] * 1024 * per["FETCH_SIZE"]["scale"]
        wb = per["WRITE_SIZE"][k][0] * 1024 * per["WRITE_SIZE"]["scale"]
        out = {"kernel": k, "workload": "batched A+B<->C: 256 x 384000-tet + 64 x 48000-tet realizations, 3 species",
               "kernel_sources": kernel_source_hash(), "bytes_per_launch": int(round(fb + wb)),
               "fetch_bytes_per_launch": int(round(fb)), "write_bytes_per_launch": int(round(wb)),
               "scale": {c: round(per[c]["scale"], 4) for c in per},
               "calibration": "bandwidth_copy_kernel copying 1 GiB reads FETCH_SIZE "
                              f"{per['FETCH_SIZE']['copy_kib']:,.0f} KiB and WRITE_SIZE "
                              f"{per['WRITE_SIZE']['copy_kib']:,.0f} KiB per dispatch",
               "launches_averaged": per["FETCH_SIZE"][k][1], "commands": command,
               "note": f"per dispatch of the last {launches} {k} launches (the single-chain timing pass, one "
                       "launch per period over all realizations); counter KiB x 1024 x scale"}
        path = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"{k}_batched_traffic.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        log(f"{path}: {out['bytes_per_launch']:.4g} B per launch")


def write_trace_summary(trace_csv, stats_csv, bench_json, launches, command, out_dir=None):
    """Turns a rocprofv3 --kernel-trace --stats run of this script into
    profiles/step_kernels_batched_trace.json: the average duration of the
    timing pass's dispatches of both step kernels (the last `launches` of each
    before the bandwidth probe's first copy), beside the averages the same run
    measured with HIP events (its JSON line, `bench_json`), and the profiler's
    per-kernel table for the whole run."""
    import csv

    rows = []
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    copies = [i for i, (_, _, n) in enumerate(rows) if "bandwidth_copy_kernel" in n]
    if not copies:
        raise SystemExit(f"no bandwidth_copy_kernel dispatch in {trace_csv}")
    pass_ids = timing_pass_ids(list(range(len(rows))), lambda i: rows[i][2], copies[0], launches, trace_csv)
    with open(bench_json) as f:
        line = json.loads([x for x in f if x.startswith("{")][-1])
    if line["config"].get("launch_shape", {}).get("fused"):
        raise SystemExit(f"{bench_json}: a fused launch shape has no scan/update timing pass")
    kern = line["roofline"]["kernels"]
    out = {"workload": "batched A+B<->C: 256 x 384000-tet + 64 x 48000-tet realizations, 3 species",
           "kernel_sources": kernel_source_hash(), "command": command, "timing_pass": {},
           "launch_shape": line["config"].get("launch_shape"), "ms_per_step": line["ms_per_step"]}
    for k in ("scan_kernel", "update_kernel"):
        ds = [rows[i] for i in pass_ids[k]]
        us = [(e - s) / 1e3 for s, e, _ in ds]
        ev = kern[k]["avg_launch_ms"] * 1e3
        avg = sum(us) / len(us)
        out["timing_pass"][k] = {"instance": ds[-1][2], "launches": len(us), "trace_avg_us": round(avg, 1),
                                 "trace_min_us": round(min(us), 1), "trace_max_us": round(max(us), 1),
                                 "hip_events_avg_us": round(ev, 1), "events_over_trace": round(ev / avg, 3)}
        log(f"{k}: trace {avg:.1f} us, HIP events {ev:.1f} us per launch over the timing pass")
    with open(stats_csv) as f:
        out["stats"] = [{"kernel": r["Name"][:120], "calls": int(r["Calls"]),
                         "average_us": round(float(r["AverageNs"]) / 1e3, 1),
                         "share_pct": round(float(r["Percentage"]), 2)}
                        for r in list(csv.DictReader(f))[:12]]
    path = os.path.join(out_dir or os.path.join(ROOT, "profiles"), "step_kernels_batched_trace.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    log(f"wrote {path}")


def update_bytes(work, species):
    """Bytes the update kernel moves for the work it counted on the device,
    in this implementation's own units:
      4 + 4 S B per queued tet (its queue entry: index and S counts),
      64 B per queued tet (its mesh record: neighbours, weights, g, N_A V),
      9 B per count addition into the next buffer (the 4 B read and 4 B
      write of the atomic, and the byte it sets in the occupancy map)."""
    return work["tets"] * (4 + 4 * species + 64) + 9 * work["additions"]


def method_bytes(work, species, mesh_tets):
    """Algorithmic bytes of the method's per-period update for the work
    counted on the device (the roofline's units): 8 B per tet-species held
    in the queue (an int32 count read and written once), 64 B per tet of
    each distinct mesh (neighbours, weights, g, N_A V), read once per period
    whatever the number of realizations sharing it, and 8 B per non-zero
    transfer across a face."""
    return 8 * species * work["tets"] + 64 * mesh_tets + 8 * work["transfers"]


def run_jittered(P, W, periods):
    """The jittered 40^3 x 6 lattice (tet volumes spanning about 4x) with
    A+B<->C and a fourth species D decaying at 1/s from 1 uM in one octant,
    run plainly (one realization); tau = tau_scale x the smallest 1/(D g)
    is about 1e-5 s here, so 0.05 s takes about 5000 periods: this runs the
    first `periods` of them, timed after a warm-up."""
    m = W.abcd_jittered()
    sim = P.Simulation.from_model(m)
    sim.step(8)
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(periods)
    sim.synchronize()
    dt = time.perf_counter() - t0
    tau = sim.tau
    # the same simulation through the engine: graph-replayed chunks of periods
    e = P.rdos_engine_create(0, 0)
    run_engine(P, e, [sim], 32)
    t1 = time.perf_counter()
    run_engine(P, e, [sim], periods)
    dte = time.perf_counter() - t1
    shape = P.rdos_engine_launch_shape(e)
    P.rdos_engine_destroy(e)
    sim.close()
    upd = periods * m.n_tets * m.n_species
    return {"workload": "jittered 40^3 x 6 Kuhn lattice (384000 tets, volumes spanning about 4x), A+B<->C plus D "
                        "decaying at 1/s from 1 uM in one octant, 4 species, 1 realization",
            "periods": periods, "tau_s": tau,
            "ms_per_period": round(dte / periods * 1e3, 5), "updates_per_s": round(upd / dte, 1),
            "engine_launch_shape": shape,
            "plain_ms_per_period": round(dt / periods * 1e3, 5), "plain_updates_per_s": round(upd / dt, 1),
            "periods_to_0.05_s": int(round(0.05 / tau)),
            "projected_s_to_0.05_s": round(dte / periods * (0.05 / tau), 4)}


def run_small_mesh(P, W):
    """The 1 um diffusion cube (750 tets, one species, 1000 molecules at the
    centre) run plainly to 0.5 s: the last period is shortened to end there
    (423 periods); a work list this small is bound by launch latency."""
    m = W.diffusion_cube()
    sim = P.Simulation.from_model(m)
    sim.run_until(m.t_end)  # warm-up pass, then the same run again from the initial state
    sim.synchronize()
    for q in range(m.n_species):
        sim.set_counts(q, m.init[0, q])
    sim.set_state(0, 0.0)
    t0 = time.perf_counter()
    sim.run_until(m.t_end)
    sim.synchronize()
    dt = time.perf_counter() - t0
    periods = sim.time()[1]
    sim.close()
    return {"workload": "1 um cube, 5^3 x 6 Kuhn lattice (750 tets), 1 species, 1000 molecules at the centre, "
                        "run to 0.5 s (422 periods + 1 shortened)", "periods": periods,
            "ms_per_period": round(dt / periods * 1e3, 5), "updates_per_s": round(periods * m.n_tets / dt, 1),
            "wall_ms": round(dt * 1e3, 3)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=338, help="timed periods (338 = 0.1 s of the A+B<->C system)")
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed periods first; the launch-shape tuner then settles in an untimed phase of its own")
    ap.add_argument("--workload", choices=["batched", "plain", "serving", "variants"], default="batched",
                    help="variants: throughput of the method options, a surface, six and ten species (not the "
                         "headline line)")
    ap.add_argument("--rate", type=float, default=20.0, help="serving: mean arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serving: seconds of arrivals")
    ap.add_argument("--request-steps", type=int, default=1000, help="serving: periods per request")
    ap.add_argument("--budget-gb", type=float, default=8.0, help="serving: HBM budget of the engine")
    ap.add_argument("--shape", default=None, metavar="CHUNK,SCAN_GRID,UPDATE_BPS,CHAINS",
                    help="batched: fix the engine's launch shape instead of tuning it (for profiled runs, where "
                         "the profiler's own cost can change the tuner's choice)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain one-realization comparison")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small-mesh (750-tet cube) and jittered-mesh (384k tets, 4 species) figures")
    ap.add_argument("--serving-seconds", type=float, default=12.0,
                    help="length of the serving leg of the default line (Poisson arrivals at --rate); 0 skips it")
    ap.add_argument("--cpu-periods", type=int, default=1014, help="oracle sample length (periods; 1014 = 0.3 s)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no run: write the kernels' HBM traffic files from two rocprofv3 --pmc runs of "
                         "`bench.py --steps K --no-cpu-baseline --no-plain` (K = --steps here)")
    ap.add_argument("--trace-from", nargs=3, metavar=("TRACE_CSV", "STATS_CSV", "BENCH_JSON"),
                    help="no run: write the step kernels' trace summary from a rocprofv3 --kernel-trace --stats "
                         "run of `bench.py --steps K --warmup W` (K, W as here) and that run's JSON line")
    ap.add_argument("--out-dir", default=None, help="with --traffic-from / --trace-from: where to write")
    args = ap.parse_args()

    def in_repo(path):
        # a path as the recorded commands name it: under $REPO, the repository root
        rel = os.path.relpath(os.path.abspath(path or "."), ROOT)
        return "$REPO" if rel == "." else ("$REPO/" + rel if not rel.startswith("..") else os.path.abspath(path))

    if args.trace_from:
        out_dir, name = os.path.split(args.trace_from[0])
        cmd = (f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
               f"-d {in_repo(out_dir)} -o {name.replace('_kernel_trace.csv', '')} -- python3 $REPO/bench.py "
               f"--gpus 1 --steps {args.steps} --warmup {args.warmup} > {in_repo(args.trace_from[2])}")
        write_trace_summary(*args.trace_from, args.steps, cmd, args.out_dir)
        return

    if args.traffic_from:
        # The timing pass is the last run of scan/update pairs only when nothing after the warm-up tunes:
        # the profiled runs fix a two-launch shape (under a profiler the tuner's choice can differ)
        if not args.shape or int(args.shape.split(",")[2]) < 1:
            raise SystemExit("--traffic-from needs the two-launch --shape the profiled runs fixed")
        # the profiler commands that wrote the two files, reconstructed from their paths
        cmd = []
        for c, csv_path in zip(("FETCH_SIZE", "WRITE_SIZE"), args.traffic_from):
            out_dir, name = os.path.split(csv_path)
            cmd.append(f"cd /tmp && export TMPDIR=/tmp && timeout -s KILL 300 rocprofv3 --pmc {c} "
                       f"--kernel-include-regex 'scan_kernel|update_kernel|bandwidth_copy' --output-format csv "
                       f"-d {in_repo(out_dir)} -o {name.replace('_counter_collection.csv', '')} -- python3 "
                       f"$REPO/bench.py --steps {args.steps} "
                       f"--warmup {args.warmup} --no-cpu-baseline --no-plain --no-small --serving-seconds 0"
                       + (f" --shape {args.shape}" if args.shape else ""))
        write_traffic(*args.traffic_from, args.steps, cmd, args.out_dir)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); realizations and requests shard "
              "across GPUs without communication, and no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    import paper_1512_03126_amd as P
    import workloads as W

    P.lib()
    K, Wm = args.steps, args.warmup
    result = {}

    if args.workload == "variants":
        res = run_variants(P, args)
        print(json.dumps({"metric": "tet-species updates/s per variant", "unit": "tet-species updates/s",
                          "n_gpus": 1, "steps": K, "warmup": Wm, "data": "synthetic", "variants": res}), flush=True)
        return

    if args.workload == "serving":
        res = run_serving(P, args)
        out = {"metric": "tet-species updates/s (served, aggregate)", "value": round(res["value"], 1),
               "unit": "tet-species updates/s", "n_gpus": 1, "steps": args.request_steps, "warmup": 0,
               "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "i32 counts / f64 probabilities", "data": "synthetic (seeded jittered lattices)",
               "config": {"workload": f"serving: Poisson {args.rate}/s for {args.duration} s, jittered Kuhn "
                                      f"lattices 1e4-1e6 tets, 1-6 species, {args.request_steps} periods each",
                          **{k: (round(v, 3) if isinstance(v, float) else v) for k, v in res.items()
                             if k != "value"}}}
        print(json.dumps(out), flush=True)
        return

    # ---------------- plain: one realization, one launch pair per period
    plain = None
    if args.workload == "plain" or not args.no_plain:
        m2 = W.abc_lattice()
        (s2,) = make_sims(P, [m2])
        s2.step(max(Wm, 1))
        s2.synchronize()
        t0 = time.perf_counter()
        s2.step(K)
        s2.synchronize()
        dt = time.perf_counter() - t0
        plain = dict(value=K * m2.n_tets * m2.n_species / dt, ms_per_step=dt / K * 1e3)
        log(f"plain A+B<->C 384k tets: {plain['value']:.3e} upd/s, {plain['ms_per_step']:.3f} ms/period")
        s2.close()

    if args.workload == "plain":
        value, ms_step = plain["value"], plain["ms_per_step"]
        workload = "A+B<->C, 40^3x6 Kuhn lattice (384000 tets x 3 species), 1 realization, one launch pair per period"
        config = {"workload": workload, "tets": 384000, "species": 3, "realizations": 1, "periods": K}
        roof = None
    else:
        log("building the batched workload (256 x 384k-tet + 64 x 48k-tet realizations)")
        models = build_batched()
        sims = make_sims(P, models)
        upd_per_period = sum(m.n_realizations * m.n_tets * m.n_species for m in models)
        bytes_per_period = 8 * upd_per_period
        mesh_tets = sum(m.n_tets for m in models)  # tets of the distinct meshes
        e = P.rdos_engine_create(0, 0)
        if args.shape:
            P.rdos_engine_set_shape(e, *(int(v) for v in args.shape.split(",")))
        if Wm > 0:
            run_engine(P, e, sims, Wm)
        # untimed: the tuner settles and the chosen shape's graph is captured
        tuning_periods = settle_engine(P, e, sims)
        shape = P.rdos_engine_launch_shape(e)
        log(f"launch shape ({shape['source']}) after {tuning_periods} untimed tuning periods: {shape}")
        tuner = [[c["chunk"], c["scan_grid"], c["update_blocks_per_segment"], c["chains"], round(c["ms_first"], 4),
                  round(c["ms_second"], 4)] for c in P.rdos_engine_tuner_scores(e)]
        if shape["source"] == "tuned":
            log("tuner (chunk, scan grid, update blocks per segment, chains, ms per period in pass 1 and 2): "
                + "; ".join(" ".join(str(v) for v in c) for c in tuner))
        st0 = P.rdos_engine_stats(e)
        t0 = time.perf_counter()
        run_engine(P, e, sims, K)
        dt = time.perf_counter() - t0
        st1 = P.rdos_engine_stats(e)
        value = K * upd_per_period / dt
        ms_step = dt / K * 1e3
        # per-kernel durations: K periods launched directly, one launch of
        # each kernel per period, none idle.  The update kernel first tallies
        # its work on the device over K periods (the tally slows it by about
        # 8%), then K more periods are timed with HIP events between the
        # launches, without the tally, as the graph replays run it; the work
        # per launch of the tallied pass stands for the timed one's (the mix
        # is stationary: its occupied tets drift by less than 0.2% over
        # hundreds of periods).  The scan's own-unit bytes are counted on the
        # state before and after the timed pass.
        P.rdos_engine_set_profiling(e, True, tally=True)
        run_engine(P, e, sims, K)
        work = P.rdos_engine_work_counts(e)
        kw = P.rdos_engine_kernel_times(e)
        alg0 = scan_bytes(sims, models)
        P.rdos_engine_set_profiling(e, True, tally=False)
        run_engine(P, e, sims, K)
        kt = P.rdos_engine_kernel_times(e)
        P.rdos_engine_set_profiling(e, False)
        alg1 = scan_bytes(sims, models)
        n_scan, n_upd = kt["scan_launches"], kt["update_launches"]
        if n_scan != K or n_upd != K or kw["update_launches"] != K:
            raise SystemExit(f"timing passes launched {kw['update_launches']} tallied updates, {n_scan} scans and "
                             f"{n_upd} updates for {K} periods")
        tallied_ms = kw["update_ms"] / K
        scan_ms = kt["scan_ms"] / n_scan
        upd_ms = kt["update_ms"] / n_upd
        log(f"batched: {value:.3e} upd/s, {ms_step:.4f} ms/period; scan {scan_ms:.4f} ms, update {upd_ms:.4f} ms "
            f"per launch ({n_upd} launches; {tallied_ms:.4f} ms while tallying); update work {work}")
        kern = {}
        for name, ms, alg in (("scan_kernel", scan_ms, 0.5 * (alg0 + alg1)),
                              ("update_kernel", upd_ms, update_bytes(work, models[0].n_species) / n_upd)):
            ach = alg / (ms * 1e-3) / 1e9
            tr = traffic_from_profile(name, "batched")
            kern[name] = {"avg_launch_ms": round(ms, 4), "own_units_bytes_per_launch": int(alg),
                          "own_units_GBps": round(ach, 1), "own_units_frac": round(ach / HBM_PEAK_GBPS, 4),
                          "traffic": tr, "traffic_GBps": round(tr / (ms * 1e-3) / 1e9, 1) if tr else None}
            log(f"{name}: {alg:.4g} B per launch in its own units, {ach:.1f} GB/s, measured traffic {tr}")
        up = kern["update_kernel"]
        up["queued_tets_per_launch"] = round(work["tets"] / n_upd, 1)
        up["additions_per_launch"] = round(work["additions"] / n_upd, 1)
        up["transfers_per_launch"] = round(work["transfers"] / n_upd, 1)
        up["avg_launch_ms_tallying"] = round(tallied_ms, 4)
        # the roofline: the update (the longer kernel) in the method's units
        alg = method_bytes(work, models[0].n_species, mesh_tets * n_upd) / n_upd
        ach = alg / (upd_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "update_kernel", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": up["traffic"],
                "algorithmic_bytes_per_launch": int(alg),
                "units": "8 B per queued tet-species + 64 B per tet of each distinct mesh + 8 B per face transfer",
                "avg_launch_ms": up["avg_launch_ms"], "kernels": kern,
                "dense_bytes_per_period": bytes_per_period,
                "dense_period_frac": round(bytes_per_period / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
        log(f"update_kernel: {alg:.4g} algorithmic B per launch (method units), {ach:.1f} GB/s, "
            f"frac {roof['frac']}")
        try:
            roof["copy_probe_GBps"] = round(P.rdos_bandwidth_probe(0, 1 << 30, 20), 1)
        except Exception as ex:  # informational only
            log(f"bandwidth probe failed: {ex}")
        # The update's count additions are random atomics into the next count
        # buffer: their rate against the device's rate for random atomics
        # alone (the same number per launch, into a buffer of the same size)
        try:
            n_add = int(up["additions_per_launch"])
            probe = P.rdos_atomic_probe(0, 4 * upd_per_period, max(n_add, 1), 10)
            up["additions_per_s"] = round(n_add / (upd_ms * 1e-3), 1)
            up["atomic_probe_per_s"] = round(probe, 1)
            up["additions_frac_of_atomic_probe"] = round(up["additions_per_s"] / probe, 4)
            log(f"update_kernel: {up['additions_per_s']:.3e} additions/s; random atomics alone "
                f"{probe:.3e}/s ({up['additions_frac_of_atomic_probe']:.2f})")
        except Exception as ex:  # informational only
            log(f"atomic probe failed: {ex}")
        P.rdos_engine_destroy(e)
        for x in sims:
            x.close()
        workload = ("batched A+B<->C: 256 realizations x 40^3x6 Kuhn lattice (384000 tets) + 64 x 20^3x6 "
                    "(48000 tets), 3 species, hipGraph-captured chunks of periods")
        config = {"workload": workload, "tets": [384000, 48000], "realizations": [256, 64], "species": 3,
                  "periods": K, "tau_s": 2.958758547680654e-4, "updates_per_period": upd_per_period,
                  "realizations_per_s": round(320.0 / (ms_step * 1e-3 * 338), 3),
                  "engine_launches_timed": st1["launches"] - st0["launches"], "launch_shape": shape,
                  "launch_shape_source": shape["source"], "tuning_periods_untimed": tuning_periods}
        if shape["source"] == "tuned":
            config["tuner_ms_per_period"] = tuner  # [chunk, scan grid, update blocks/segment, chains, pass 1, 2]
        if plain:
            config["plain_updates_per_s"] = round(plain["value"], 1)
            config["plain_ms_per_step"] = round(plain["ms_per_step"], 4)
            config["batched_over_plain"] = round(value / plain["value"], 2)

    small = jittered = None
    if not args.no_small:
        small = run_small_mesh(P, W)
        log(f"small mesh: {small['ms_per_period']:.4f} ms/period ({small['periods']} periods)")
        jittered = run_jittered(P, W, 400)
        log(f"jittered A+B<->C + D: {jittered['updates_per_s']:.3e} upd/s, {jittered['ms_per_period']:.4f} ms/period "
            f"through the engine ({jittered['plain_ms_per_period']:.4f} plainly)")

    served = None
    if args.serving_seconds > 0:
        sargs = argparse.Namespace(seed=args.seed, rate=args.rate, duration=args.serving_seconds,
                                   request_steps=args.request_steps, budget_gb=args.budget_gb)
        res = run_serving(P, sargs)
        served = {"workload": f"Poisson {args.rate}/s arrivals for {args.serving_seconds:g} s, jittered Kuhn lattices "
                              f"1e4-1e6 tets (log-uniform), 1-6 species, random reactions, "
                              f"{args.request_steps} periods each, HBM budget {args.budget_gb:g} GB",
                  **{k: (round(v, 3) if isinstance(v, float) else v) for k, v in res.items()}}
        served["updates_per_s"] = served.pop("value")

    cpu = None
    if not args.no_cpu_baseline:
        m2 = W.abc_lattice()
        v1, dt1 = oracle_baseline(m2, args.cpu_periods)
        log(f"cpu oracle, one thread: {v1:.3e} upd/s over {dt1:.1f} s")
        threads = min(cpu_cores(), 16)
        pt = max(args.cpu_periods // 4, 1)
        vt, dtt = oracle_baseline_threads(m2, pt, threads)
        log(f"cpu oracle, {threads} threads: {vt:.3e} upd/s over {dtt:.1f} s")
        cpu = {"value": round(vt, 1), "unit": "tet-species updates/s", "cores": threads, "kind": "oracle",
               "sample": f"A+B<->C 40^3x6 (384000 tets x 3 species): {threads} realizations on {threads} threads, "
                         f"{pt} periods each ({dtt:.1f} s wall); one thread alone, 1 realization x "
                         f"{args.cpu_periods} periods: {v1:.4g} updates/s ({dt1:.1f} s). {cpu_model()}, "
                         f"{cpu_cores()} cores available",
               "single_thread_value": round(v1, 1)}

    out = {"metric": "tet-species updates/s", "value": round(value, 1), "unit": "tet-species updates/s",
           "n_gpus": 1, "steps": K, "warmup": Wm, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "i32 counts / f64 probabilities",
           "data": "synthetic (seeded Kuhn lattices, molecules placed by volume)", "config": config}
    if roof:
        out["roofline"] = roof
    if cpu:
        out["cpu_baseline"] = cpu
    if served:
        out["serving"] = served
    if small:
        out["small_mesh"] = small
    if jittered:
        out["jittered_mesh"] = jittered
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
