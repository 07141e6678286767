"""Benchmark: devices evaluated and stamped per second for one Newton-Raphson step.

Workload (default): inverter chain of 100,000 stages (200,000 MOSFETs, 100,003 MNA
rows, 500,006 nonzeros), rail-excluded conflict rule (4 colours), FP64, one NR step
= evaluate every device at x and stamp A, b (ag0 = 1e12, backward Euler with h = 1
ps).  Synthetic seeded inputs (W, L, VTH0, x).  Every variant is timed as K replays
of a HIP graph holding one step; the headline variant also as K launches back to
back on the stream, and the faster of the two gives `value`.

Prints one JSON line.  Extra keys report the other kernel variants, the 6T SRAM
array, the batched sweep and the adjoint, plus the roofline of the dominant kernel
and the oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP64_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x FP64 lanes x clock: one op per lane-cycle
KERNEL_OF = {"persistent": "k_persistent_* (one launch per step)",
             "region": "k_region + k_region_tail (one launch each per step)",
             "per_kernel": "k_colour_phase x colours + k_hub",
             "buffered": "k_eval_buffer + k_persistent_stamp",
             "atomic": "k_fill_zero + k_atomic",
             "atomic_wave": "k_fill_zero + k_atomic_wave (hub entries summed per wave)",
             "serial": "k_fill_zero + k_eval_buffer + k_serial_stamp (one lane)"}
PEAK_HBM = 8.0e12
AG0 = 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2604_03079_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def device_tensors(torch, circ, dev):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t(circ.W), t(circ.L), t(circ.VTH0), t(circ.x)


def release(torch, *handles):
    """Finish the device work, then destroy library handles now, while the HIP runtime
    (and a profiler attached to it) is alive, instead of at interpreter exit."""
    torch.cuda.synchronize()
    for h in handles:
        h.close()


def time_graph(torch, fn, steps, warmup):
    """Capture fn() (one NR step) in a graph; replay warmup times, then time steps."""
    fn()
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, g


def time_eager(torch, fn, steps, warmup):
    """Average duration of fn() launched back to back on the current stream, between
    two events on that stream (the kernel's own time plus launch gaps)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_cold(torch, fn, steps, flush_mib=512):
    """Median duration of fn() with a flush of flush_mib MiB written to HBM before each
    step (outside the timed interval), so that no input is cache resident."""
    flush = torch.empty(flush_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for i, (e0, e1) in enumerate(ev):
        flush.fill_(float(i))
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))


def algorithmic_counts(circ, exclude=True):
    """FP64 operations and bytes of one step of the coloured method (counted on the
    oracle's definition of the step).

    ops: the oracle's operation counter over model M (+, -, *, /, sqrt each one)
    less its size-dependent constants (computed once per parameter set, when the
    parameters are set, not per step), plus the merge adds of devices with coinciding
    terminals, one add per load-add stamp and the hub sums' adds.
    method_bytes: the fused coloured method's own HBM traffic per step, itemised per
    device: the nine per-device model constants and the polarity (73 B), four terminal
    indices (16 B), x read once (8 B per row), one 4-byte stamp code per matrix
    slot-write, an 8-byte store per matrix slot-write, an 8-byte read per load-add
    (slot-writes beyond the first writer of each entry), the same store and read terms
    for the RHS writes, and for the hub entries one part per 32 contributions (summed
    on chip), written and read back (16 B per part).
    floor_bytes: inputs once and outputs once (context only)."""
    from oracle import oracle as O
    from paper_2604_03079_amd import netgen as G
    rp, ci = O.pattern(circ)
    col, C, _ = O.colour(circ, exclude)
    O.lib().or_count_ops(1)
    O.assemble(circ, rp, ci, G.default_card(1), G.default_card(-1), AG0, col=col, exclude=exclude)
    model_ops = O.lib().or_ops()
    O.lib().or_count_ops(0)
    # the size-dependent share is the same for every device (no branches)
    sizedep = O.model_sizedep_opcount(G.default_card(1), 1, 1e-6, 45e-9, 0.4, [0.5, 0.5, 0.0, 0.0])
    model_ops -= sizedep * circ.n_dev
    slot, sflag, brow, bflag = O.stamp_map(circ, rp, ci, col, exclude)
    merges = 0
    for t4 in circ.term:
        nz = [int(n) for n in t4 if n != 0]
        k = len(set(nz))
        merges += len(nz) * len(nz) - k * k + len(nz) - k
    add_ops = int((sflag == 0).sum() + (bflag == 0).sum())
    hub_sizes = {}
    for s_ in slot[sflag == 2]:
        hub_sizes[("A", int(s_))] = hub_sizes.get(("A", int(s_)), 0) + 1
    for r in brow[bflag == 2]:
        hub_sizes[("b", int(r))] = hub_sizes.get(("b", int(r)), 0) + 1
    hub_ops = sum(m - 1 for m in hub_sizes.values())
    ops = model_ops + merges + add_ops + hub_ops
    n = circ.n_dev
    nslot = int((sflag >= 0).sum())
    nbrow = int((bflag >= 0).sum())
    slots_written = int(np.unique(slot[sflag >= 0]).size)
    rows_written = int(np.unique(brow[bflag >= 0]).size)
    hub_parts = sum((m + 31) // 32 for m in hub_sizes.values())
    items = dict(device_constants=73 * n, terminals=16 * n, x=8 * circ.n_rows, stamp_codes=4 * nslot,
                 A_stores=8 * nslot, A_load_add_reads=8 * (nslot - slots_written),
                 b_stores=8 * nbrow, b_load_add_reads=8 * (nbrow - rows_written), hub_parts=16 * hub_parts)
    floor = n * (24 + 1 + 16) + 8 * circ.n_rows + 4 * (nslot + nbrow) + 8 * len(ci) + 8 * circ.n_rows
    return dict(ops=int(ops), model_ops=int(model_ops), method_bytes=int(sum(items.values())),
                method_bytes_items=items, floor_bytes=int(floor), n_colors=int(C), n_dev=int(n))


def add_counts(parts):
    """Sum of algorithmic_counts over the circuits of a batch."""
    out = dict(ops=0, model_ops=0, method_bytes=0, floor_bytes=0, n_dev=0, n_colors=0, method_bytes_items={})
    for p in parts:
        for k in ("ops", "model_ops", "method_bytes", "floor_bytes", "n_dev"):
            out[k] += p[k]
        out["n_colors"] = max(out["n_colors"], p["n_colors"])
        for k, v in p["method_bytes_items"].items():
            out["method_bytes_items"][k] = out["method_bytes_items"].get(k, 0) + v
    return out


def roofline(counts, kernel_ms, traffic, kernel):
    """Roofline of one step against its binding resource: t_FP64 = ops / FP64 lane-op
    peak, t_HBM = method bytes / HBM peak; the larger is the bound, frac = that time
    over the measured kernel time."""
    secs = kernel_ms * 1e-3
    t_fp64 = counts["ops"] / PEAK_FP64_OPS
    t_hbm = counts["method_bytes"] / PEAK_HBM
    common = dict(traffic=traffic, t_fp64_us=round(t_fp64 * 1e6, 3), t_hbm_us=round(t_hbm * 1e6, 3),
                  kernel_avg_us=round(kernel_ms * 1e3, 3), kernel=kernel,
                  algorithmic_ops_per_launch=counts["ops"], method_bytes_per_launch=counts["method_bytes"],
                  method_bytes_per_device=round(counts["method_bytes"] / counts["n_dev"], 2),
                  fp64_op_frac=round(t_fp64 / secs, 5), hbm_frac=round(t_hbm / secs, 5),
                  floor_bytes_per_launch_context=counts["floor_bytes"])
    if t_hbm >= t_fp64:
        ach = counts["method_bytes"] / secs / 1e9
        return dict(bound="hbm", achieved=round(ach, 2), peak=PEAK_HBM / 1e9, unit="GB/s",
                    frac=round(t_hbm / secs, 5), **common)
    ach = counts["ops"] / secs / 1e12
    return dict(bound="alu", achieved=round(ach, 4), peak=round(PEAK_FP64_OPS / 1e12, 2),
                unit="T FP64 op/s", frac=round(t_fp64 / secs, 5), **common)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(circ, budget_s=10.0):
    """The oracle on the host, same inputs: the serial colour replay on one core (the
    paper's single-thread loadsingle form), then the colour replay spread over every
    OpenMP thread (the paper's ColorFused on its CPU), which must give the same bits.
    Devices per second of each; `value` is the all-core leg."""
    from oracle import oracle as O
    from paper_2604_03079_amd import netgen as G
    rp, ci = O.pattern(circ)
    col, _, _ = O.colour(circ, True)
    nc, pc = G.default_card(1), G.default_card(-1)
    legs = {}
    outs = {}
    for key, threads in (("serial_one_core", False), ("colour_replay_all_threads", True)):
        it = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s or it < 3:
            outs[key] = O.assemble(circ, rp, ci, nc, pc, AG0, col=col, exclude=True, threads=threads)
            it += 1
        dt = time.perf_counter() - t0
        legs[key] = dict(value=round(circ.n_dev * it / dt / 1e6, 4), unit="M devices/s",
                         cores=O.omp_threads() if threads else 1, steps=it, seconds=round(dt, 2))
    same = all(np.array_equal(a.view(np.int64), b.view(np.int64))
               for a, b in zip(outs["serial_one_core"], outs["colour_replay_all_threads"]))
    main = legs["colour_replay_all_threads"]
    return dict(value=main["value"], unit="M devices/s", cores=main["cores"], kind="oracle",
                host=f"{cpu_model()}, {os.cpu_count()} logical CPUs visible",
                sample=f"full {circ.n_dev}-device chain, colour replay (C, -O2): {main['steps']} steps on "
                       f"{main['cores']} OpenMP threads; serial leg {legs['serial_one_core']['steps']} steps on 1 core",
                legs=legs, threaded_bits_equal_serial=bool(same))


def traffic_from_profiles(kernel_hash: str, key: str):
    p = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        d = json.load(open(p))
    except Exception:
        return None
    e = d.get(key)
    if not e or e.get("kernel_hash") != kernel_hash:
        return None
    return e.get("bytes_per_launch")


def summarize_pmc(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, kernel, key, copy_mib):
    """HBM bytes per launch of `kernel` from two rocprofv3 --pmc runs (FETCH_SIZE,
    WRITE_SIZE; KiB per dispatch), each scaled by what the same counter reads for a
    plain device copy of copy_mib MiB; written to profiles/hbm_traffic.json."""
    import csv

    def base(kernel_name):   # "void cs::k_region<false>(cs::KCirc, ...)" -> "void cs::k_region"
        head = kernel_name.split("(")[0]
        return head[:head.index("<")] if "<" in head else head

    def per_dispatch(path, name, counter):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                if base(r["Kernel_Name"]).endswith(name) and r["Counter_Name"] == counter]
        return sum(vals) / len(vals), len(vals)

    # the kernels of one step: their per-dispatch averages add up
    kf = kw = 0.0
    nf = nw = 0
    for name in kernel.split(","):
        f_, n_ = per_dispatch(fetch_csv, name, "FETCH_SIZE")
        w_, m_ = per_dispatch(write_csv, name, "WRITE_SIZE")
        kf, kw, nf, nw = kf + f_, kw + w_, max(nf, n_), max(nw, m_)
    cf, _ = per_dispatch(copy_fetch_csv, "__amd_rocclr_copyBuffer", "FETCH_SIZE")
    cw, _ = per_dispatch(copy_write_csv, "__amd_rocclr_copyBuffer", "WRITE_SIZE")
    copy_bytes = copy_mib * (1 << 20)
    ff, wf = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    entry = dict(kernel=kernel, kernel_hash=kernel_sources_hash(), dispatches=[nf, nw],
                 fetch_kib=round(kf, 1), write_kib=round(kw, 1), copy_mib=copy_mib,
                 copy_fetch_kib=round(cf, 1), copy_write_kib=round(cw, 1),
                 fetch_factor=round(ff, 4), write_factor=round(wf, 4),
                 bytes_per_launch=int(kf * 1024 * ff + kw * 1024 * wf))
    p = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    d = json.load(open(p)) if os.path.exists(p) else {}
    d[key] = entry
    with open(p, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(entry))


def bench_junction_level(torch, CS, G, dev):
    """The second model level (source/drain-body junctions on every FET) on the
    chain of 100,000 stages: the region step against model M's."""
    circ = G.workload(1)
    W, L, V, x = device_tensors(torch, circ, dev)
    out = dict(n_dev=circ.n_dev)
    for key, nm, pm in (("model_m", G.default_card(1), G.default_card(-1)),
                        ("with_junctions", G.junction_card(1), G.junction_card(-1))):
        c = CS.prepare(circ, exclude=True, nmos=nm, pmos=pm)
        c.set_params(W, L, V)
        A = torch.empty(c.nnz, dtype=torch.float64, device=dev)
        b = torch.empty(c.n_rows, dtype=torch.float64, device=dev)
        step = lambda: c.eval_stamp(x, AG0, None, A, b, "region")
        ms_g, g = time_graph(torch, step, 50, 5)
        ms_s = time_eager(torch, step, 50, 5)
        ms = min(ms_g, ms_s)
        c.check()
        out[key] = dict(ms_per_step=round(ms, 5), value=round(circ.n_dev / ms / 1e3, 2),
                        graph_ms_per_step=round(ms_g, 5), stream_ms_per_step=round(ms_s, 5))
        del g
        release(torch, c)
    out["junction_cost"] = round(out["with_junctions"]["ms_per_step"] / out["model_m"]["ms_per_step"], 3)
    out["launch"] = "faster of graph replay and stream launches, per model"
    log(f"  junction level, chain100k region: {out['with_junctions']['ms_per_step'] * 1e3:.1f} us "
        f"({out['junction_cost']} x model M's {out['model_m']['ms_per_step'] * 1e3:.1f} us; graph "
        f"{out['model_m']['graph_ms_per_step'] * 1e3:.1f} / {out['with_junctions']['graph_ms_per_step'] * 1e3:.1f} us, "
        f"stream {out['model_m']['stream_ms_per_step'] * 1e3:.1f} / {out['with_junctions']['stream_ms_per_step'] * 1e3:.1f} us)")
    return out


def bench_newton(torch, CS, G, dev):
    """The Newton loop the stamp serves: one backward-Euler step (ag0 = 1e12, history
    terms N(0, 1e-5)) of the 100,000-stage chain with its input held at 0.3 V, and of
    the 64-bit adder with every net split by its 5,696 series resistors (Table I's
    R89 shape), from the generators' start points.  Per iteration: the stamp (region
    variant), the refactorisation (fused with the forward substitution for the
    level-scheduled kernels) and solve, the update, for this library's solver and
    rocSOLVER's; the first call's host factorisation is reported apart."""
    out = {}
    for key, circ in (("chain100k_be", G.chain_dc_case(100_000, 2, 0.3)),
                      ("adder64_r89_be", G.adder_case(64, 9, "all"))):
        hist = torch.from_numpy(np.random.default_rng(14).normal(0, 1e-5, (circ.n_dev, 4))).to(dev)
        c = CS.prepare(circ, exclude=True)
        W, L, V, x0 = device_tensors(torch, circ, dev)
        c.set_params(W, L, V)
        row = dict(n_dev=circ.n_dev, n_res=circ.n_res, n_rows=c.n_rows, nnz=c.nnz)
        for solver in ("levels", "rocsolver"):
            x = x0.clone()
            first = c.newton(x, AG0, hist, solver=solver)    # factor pattern, analysis
            x = x0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = c.newton(x, AG0, hist, solver=solver)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
            c.check()
            it = max(r["iterations"], 1)
            per = {k: round(v / it, 4) for k, v in r["ms"].items() if k != "host_factor"}
            row[solver] = dict(iterations=r["iterations"], converged=r["converged"], ms_per_iteration=per,
                               wall_ms=round(wall, 3),
                               solve_over_stamp=round((per["refactor"] + per["solve"]) / per["stamp"], 1))
            row["host_factor_ms"] = round(first["ms"]["host_factor"], 2)
            log(f"  newton {key} {solver}: {r['iterations']} iterations, per iteration stamp {per['stamp']:.3f} ms, "
                f"refactor {per['refactor']:.3f} ms, solve {per['solve']:.3f} ms, update {per['update']:.3f} ms; "
                f"wall {wall:.1f} ms")
        out[key] = row
    # a backward-Euler transient of the chain: 20 steps of 1 ps (history terms from
    # the charges at each step's start, then the Newton loop), level-scheduled solver
    circ = G.chain_dc_case(100_000, 2, 0.3)
    c = CS.prepare(circ, exclude=True)
    W, L, V, x0 = device_tensors(torch, circ, dev)
    c.set_params(W, L, V)
    x = x0.clone()
    c.transient(x, 1e-12, 1)                      # factor pattern and analysis
    x = x0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, iters = c.transient(x, 1e-12, 20)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    out["chain100k_transient_20_steps"] = dict(h_s=1e-12, steps=20, total_ms=round(ms, 2),
                                               ms_per_step=round(ms / 20, 3), newton_iterations=iters)
    log(f"  transient chain100k: 20 steps of 1 ps in {ms:.1f} ms ({ms / 20:.2f} ms per step), "
        f"Newton iterations {iters}")
    out["adder64_r89_sizing_batch"] = bench_batch_newton(torch, CS, G, dev)
    return out


def bench_batch_newton(torch, CS, G, dev, n_var=32):
    """A sizing loop's batch (the paper's motivation): n_var parameter draws of the
    split 64-bit adder, one backward-Euler Newton solve of all of them at once
    (cs_batch_newton, block-diagonal system) against one cs_newton per variant with
    the faster single-circuit solver, after every factorisation is made."""
    variants = [G.adder_case(64, 100 + k, "all") for k in range(n_var)]
    cs = [CS.prepare(v, exclude=True) for v in variants]
    B = CS.Batch(cs)
    B.set_launch(block=256, schedule="region")    # the batched stamp's tuned schedule
    cat = lambda a: torch.from_numpy(np.concatenate([getattr(v, a) for v in variants])).to(dev)
    W, L, V, x0 = cat("W"), cat("L"), cat("VTH0"), cat("x")
    B.set_params(W, L, V)
    hist = torch.from_numpy(np.random.default_rng(15).normal(0, 1e-5, (B.n_dev, 4))).to(dev)
    row = dict(n_variants=n_var, n_dev=B.n_dev, n_rows=B.n_rows, nnz=B.nnz)
    for solver in ("levels", "rocsolver"):
        first = B.newton(x0.clone(), AG0, hist, solver=solver)
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = B.newton(x, AG0, hist, solver=solver)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        B.check()
        it = max(r["iterations"], 1)
        row["batch_" + solver] = dict(iterations=r["iterations"], converged=r["converged"], wall_ms=round(wall, 3),
                                      ms_per_iteration={k: round(v / it, 4) for k, v in r["ms"].items()
                                                        if k != "host_factor"},
                                      host_factor_ms=round(first["ms"]["host_factor"], 2))
        log(f"  sizing batch {n_var} x adder64 R89 {solver}: {r['iterations']} iterations, wall {wall:.1f} ms "
            f"({wall / n_var:.2f} ms per variant), host factorisation {first['ms']['host_factor']:.0f} ms")
    B.per_circuit_params(W, L, V)
    xs, hs = [], []
    for i, c in enumerate(cs):
        r0, r1 = int(B.row_off[i]), int(B.row_off[i + 1])
        a, z = int(B.dev_off[i]), int(B.dev_off[i + 1])
        xs.append((r0, r1))
        hs.append(hist[a:z])
        c.newton(x0[r0:r1].clone(), AG0, hs[-1], solver="rocsolver")   # factor pattern, analysis
    x = x0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = [c.newton(x[r0:r1], AG0, h, solver="rocsolver")["iterations"] for c, (r0, r1), h in zip(cs, xs, hs)]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    row["per_variant_rocsolver"] = dict(wall_ms=round(wall, 3), iterations=its)
    best = min(row["batch_levels"]["wall_ms"], row["batch_rocsolver"]["wall_ms"])
    row["speedup_batch_vs_per_variant"] = round(wall / best, 2)
    log(f"  sizing batch: one cs_newton per variant (rocSOLVER) {wall:.1f} ms; batch {wall / best:.1f} x faster")
    return row


def bench_batch(torch, CS, G, dev):
    """512 uneven circuits: autotuned batched kernel vs one launch per circuit."""
    from paper_2604_03079_amd import autotune
    t0 = time.perf_counter()
    circs = G.workload(3)
    cs = [CS.prepare(c, exclude=True) for c in circs]
    B = CS.Batch(cs)
    setup_s = time.perf_counter() - t0
    cat = lambda a: torch.from_numpy(np.concatenate([getattr(c, a) for c in circs])).to(dev)
    W, L, V, x = cat("W"), cat("L"), cat("VTH0"), cat("x")
    A = torch.empty(B.nnz, dtype=torch.float64, device=dev)
    b = torch.empty(B.n_rows, dtype=torch.float64, device=dev)
    best = autotune.tune(B, W, L, V, x, AG0, A, b, cache_path=None, reps=5, log=log)
    ms_b, _ = time_graph(torch, lambda: B.eval_stamp(x, AG0, None, A, b), 20, 3)
    ms_e = time_eager(torch, lambda: B.eval_stamp(x, AG0, None, A, b), 20, 3)
    B.check()
    counts = add_counts([algorithmic_counts(c) for c in circs])
    roof = roofline(counts, ms_e, traffic_from_profiles(kernel_sources_hash(), "batch512"),
                    "k_region + k_region_tail (one launch each per batched step)" if best["schedule"] == "region"
                    else "k_persistent_* (one launch per batched step)")
    log(f"  batch 512 roofline: {roof['bound']} {roof['achieved']} {roof['unit']} = {roof['frac']:.3f} of peak "
        f"(t_FP64 {roof['t_fp64_us']} us, t_HBM {roof['t_hbm_us']} us, kernel {roof['kernel_avg_us']} us)")
    # adjoint of the batched step: cotangents N(0,1) on every circuit's A and b
    Ab, bb = G.cotangents(B.nnz, B.n_rows, seed=50)
    Ab, bb = torch.from_numpy(Ab).to(dev), torch.from_numpy(bb).to(dev)
    ms_a, _ = time_graph(torch, lambda: B.vjp(x, AG0, Ab, bb), 20, 3)
    ms_as = time_eager(torch, lambda: B.vjp(x, AG0, Ab, bb), 20, 3)
    B.check()
    log(f"  batch 512: adjoint {ms_a:.3f} ms ({ms_a / ms_b:.2f} x the batched forward; stream {ms_as:.3f} ms, "
        f"{ms_as / ms_e:.2f} x)")
    B.per_circuit_params(W, L, V)
    ms_p, _ = time_graph(torch, lambda: B.per_circuit_eval(x, AG0, A, b), 5, 1)
    log(f"  batch 512: batched {ms_b:.3f} ms ({B.n_dev / ms_b / 1e3:.1f} M dev/s), "
        f"per-circuit launches {ms_p:.3f} ms ({B.n_dev / ms_p / 1e3:.1f} M dev/s), setup {setup_s:.1f} s")
    return dict(n_circuits=len(circs), n_dev=B.n_dev, n_rows=B.n_rows, nnz=B.nnz,
                max_colors=B.info()["max_colors"], tuned=best, roofline=roof,
                batched=dict(ms_per_step=round(ms_b, 4), value=round(B.n_dev / ms_b / 1e3, 2),
                             stream_ms_per_step=round(ms_e, 4)),
                per_circuit_launches=dict(ms_per_step=round(ms_p, 4), value=round(B.n_dev / ms_p / 1e3, 2)),
                speedup_batched_vs_per_circuit=round(ms_p / ms_b, 2), host_setup_s=round(setup_s, 2),
                adjoint=dict(ms_per_step=round(ms_a, 4), adjoint_over_forward=round(ms_a / ms_b, 3),
                             stream_ms_per_step=round(ms_as, 4), stream_adjoint_over_forward=round(ms_as / ms_e, 3)))


def bench_adder(torch, CS, G, dev):
    """The paper's benchmark shape: a 64-bit ripple-carry adder of 28-transistor
    mirror cells (1,792 FETs), under the paper's conflict rule (896 colours, Table I),
    with the rail excluded, and with every net split by series resistors (Table I's
    R89 row: one colour); every variant, one NR step each."""
    out = dict(n_dev=1792)
    for key, split, excl in (("paper_rule", None, False), ("rails_excluded", None, True),
                             ("r89_split_paper_rule", "all", False)):
        circ = G.adder_case(64, seed=9, split=split)
        W, L, V, x = device_tensors(torch, circ, dev)
        row = {}
        for variant in ("region", "persistent", "per_kernel", "buffered", "atomic", "atomic_wave", "serial"):
            c = CS.prepare(circ, exclude=excl)
            c.set_params(W, L, V)
            A = torch.empty(c.nnz, dtype=torch.float64, device=dev)
            b = torch.empty(c.n_rows, dtype=torch.float64, device=dev)
            steps = 3 if variant == "serial" else 20
            ms, _ = time_graph(torch, lambda: c.eval_stamp(x, AG0, None, A, b, variant), steps, 2)
            c.check()
            row[variant] = dict(ms_per_step=round(ms, 5), value=round(circ.n_dev / ms / 1e3, 2))
            row["n_colors"] = c.info()["n_colors"]
        out[key] = row
        log(f"  adder 64x28T {key:20s} C {row['n_colors']:4d}: " +
            ", ".join(f"{v} {row[v]['ms_per_step'] * 1e3:.1f} us" for v in
                      ("region", "persistent", "per_kernel", "buffered", "atomic", "atomic_wave", "serial")))
    return out


SWEEP_GROUPS = (1, 2, 4, 8, 16, 32, 64, 128, 256)
SWEEP_SIZES = (200_000, 2_000)
SWEEP_MAX_PHASES = 5000   # per-colour and phase-only persistent runs above this are not timed


def bench_csweep(torch, CS, G, dev, steps=20):
    """Colour-count sweep: parallel-inverter chains (group g inverters per stage, so
    adjacent stages form a clique of 4g devices and the rail-excluded colouring needs
    4g colours) at about 200,000 and 2,000 devices, then the plain chain with the rail
    excluded or not (4 colours vs one per PMOS plus one).  Every variant per point."""
    cases = []
    for n in SWEEP_SIZES:
        for g in SWEEP_GROUPS:
            cases.append((f"pchain_n{n}_g{g}", lambda n=n, g=g: G.pchain_case(n, g, seed=7), True))
    for n in SWEEP_SIZES:
        for excl in (True, False):
            cases.append((f"chain_n{n}_{'excl' if excl else 'strict'}",
                          lambda n=n: G.chain_case(n // 2, seed=8), excl))
    out = []
    for name, make, excl in cases:
        circ = make()
        W, L, V, x = device_tensors(torch, circ, dev)
        row = dict(case=name, n_dev=circ.n_dev, rails_excluded=excl)
        for variant in ("region", "persistent", "per_kernel", "atomic", "atomic_wave"):
            c = CS.prepare(circ, exclude=excl)
            row["n_colors"] = c.info()["n_colors"]
            many = row["n_colors"] > SWEEP_MAX_PHASES
            if variant == "per_kernel" and many:
                row[variant] = None
                continue
            # above the phase limit the persistent variant runs only in its grid-barrier
            # form (every region resident), never as one grid phase per colour
            c.set_launch(256, 1 if many else -1, True)
            c.set_params(W, L, V)
            A = torch.empty(c.nnz, dtype=torch.float64, device=dev)
            b = torch.empty(c.n_rows, dtype=torch.float64, device=dev)
            try:
                ms, _ = time_graph(torch, lambda: c.eval_stamp(x, AG0, None, A, b, variant), steps, 3)
            except CS.CsError as e:
                log(f"  {name} {variant}: {e}")
                row[variant] = None
                continue
            c.check()
            row[variant] = dict(ms_per_step=round(ms, 5), value=round(circ.n_dev / ms / 1e3, 2))
            if variant == "persistent":
                row[variant]["grid_barrier_form"] = c.info()["eval_ahead"] == 1
        fmt = lambda v: f"{row[v]['value']:9.1f}" if row[v] else "        -"
        log(f"  {name:24s} n_dev {circ.n_dev:7d} C {row['n_colors']:6d}  M dev/s: region {fmt('region')} "
            f"persistent {fmt('persistent')} per-colour {fmt('per_kernel')} atomic {fmt('atomic')}")
        out.append(row)
    return out


def bench_adjoint(torch, CS, G, dev):
    """Forward + hand-written adjoint: chain of 10,000 stages, cotangents N(0,1)."""
    circ = G.workload(4)
    c = CS.prepare(circ, exclude=True)
    W, L, V, x = device_tensors(torch, circ, dev)
    c.set_params(W, L, V)
    Ab, bb = G.cotangents(c.nnz, c.n_rows, seed=50)
    Ab, bb = torch.from_numpy(Ab).to(dev), torch.from_numpy(bb).to(dev)
    A = torch.empty(c.nnz, dtype=torch.float64, device=dev)
    b = torch.empty(c.n_rows, dtype=torch.float64, device=dev)
    # both legs timed as graph replays and as stream launches; each takes the faster
    # (at 20,000 devices a kernel lasts about as long as a launch)
    fwd = lambda: c.eval_stamp(x, AG0, None, A, b, "region")
    adj = lambda: c.vjp(x, AG0, Ab, bb)
    ms_fg, _ = time_graph(torch, fwd, 50, 5)
    ms_ag, _ = time_graph(torch, adj, 50, 5)
    ms_fs = time_eager(torch, fwd, 50, 5)
    ms_as = time_eager(torch, adj, 50, 5)
    ms_f, ms_a = min(ms_fg, ms_fs), min(ms_ag, ms_as)
    log(f"  adjoint chain10k: forward {ms_f * 1e3:.1f} us, adjoint {ms_a * 1e3:.1f} us, ratio {ms_a / ms_f:.2f} "
        f"(graph {ms_fg * 1e3:.1f} / {ms_ag * 1e3:.1f} us, stream {ms_fs * 1e3:.1f} / {ms_as * 1e3:.1f} us)")
    # the paper's four evaluation-kernel variants on the same step: serial stamping
    # after a parallel evaluation (loadomp), buffered evaluation then colour phases
    # (Color), and the fused coloured schedule (ColorFused: region)
    ms_b, _ = time_graph(torch, lambda: c.eval_stamp(x, AG0, None, A, b, "buffered"), 20, 3)
    ms_s, _ = time_graph(torch, lambda: c.eval_stamp(x, AG0, None, A, b, "serial"), 3, 1)
    c.check()
    log(f"  chain10k: serial stamp (loadomp) {ms_s * 1e3:.1f} us, buffered (Color) {ms_b * 1e3:.1f} us, "
        f"region {ms_f * 1e3:.1f} us")
    return dict(workload="inverter_chain_10k_stages", n_dev=circ.n_dev,
                forward_ms=round(ms_f, 5), adjoint_ms=round(ms_a, 5),
                adjoint_over_forward=round(ms_a / ms_f, 3),
                launch="faster of graph replay and stream launches, per leg",
                graph=dict(forward_ms=round(ms_fg, 5), adjoint_ms=round(ms_ag, 5)),
                stream=dict(forward_ms=round(ms_fs, 5), adjoint_ms=round(ms_as, 5)),
                forward_plus_adjoint_value=round(circ.n_dev / (ms_f + ms_a) / 1e3, 2),
                variants_ms=dict(serial_stamp=round(ms_s, 5), buffered=round(ms_b, 5), region=round(ms_f, 5)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--variant", default="region")
    ap.add_argument("--no-extras", action="store_true", help="skip SRAM/batch/adjoint lines")
    ap.add_argument("--no-cpu", action="store_true", help="skip the host oracle timing")
    ap.add_argument("--only", action="store_true", help="time only --variant (profiling runs)")
    ap.add_argument("--ordinary", action="store_true",
                    help="with --only: launch grid-barrier kernels without the cooperative launch API")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB ten times (HBM counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write profiles/hbm_traffic.json from rocprofv3 counter CSVs and exit")
    ap.add_argument("--csweep", action="store_true",
                    help="run only the colour-count sweep and print it as one JSON line")
    ap.add_argument("--newton", action="store_true",
                    help="run only the Newton-loop leg (stamp, refactorisation, solve) and print its JSON")
    ap.add_argument("--sram-only", action="store_true",
                    help="time only the 256 x 256 SRAM's region step (profiling runs)")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the 512-circuit batched step (region schedule, block 256) and its adjoint (profiling runs)")
    ap.add_argument("--pmc-kernel", default="k_region,k_region_tail",
                    help="kernels of one step (comma-separated) whose counters --summarize-pmc sums")
    ap.add_argument("--pmc-key", default="region_chain100k")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.pmc_kernel, args.pmc_key, 256)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: every box here has one GPU (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_03079_amd import colorstamp as CS
    from paper_2604_03079_amd import netgen as G

    dev = torch.device("cuda:0")
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 10 copies of {args.copy_probe} MiB")
        return
    if args.newton:
        print(json.dumps({"newton": bench_newton(torch, CS, G, dev), "kernel_sources": kernel_sources_hash()}),
              flush=True)
        return
    if args.sram_only:
        sram = G.workload(2)
        c = CS.prepare(sram, exclude=True)
        Ws, Ls, Vs, xs = device_tensors(torch, sram, dev)
        c.set_params(Ws, Ls, Vs)
        A = torch.empty(c.nnz, dtype=torch.float64, device=dev)
        b = torch.empty(c.n_rows, dtype=torch.float64, device=dev)
        ms = time_eager(torch, lambda: c.eval_stamp(xs, AG0, None, A, b, "region"), args.steps, args.warmup)
        c.check()
        log(f"sram 256x256 region block 256: {ms * 1e3:.1f} us per step ({args.steps} steps)")
        release(torch, c)
        return
    if args.batch_only:
        circs = G.workload(3)
        B = CS.Batch([CS.prepare(c, exclude=True) for c in circs])
        B.set_launch(256, -1, 0, schedule="region")
        cat = lambda a: torch.from_numpy(np.concatenate([getattr(c, a) for c in circs])).to(dev)
        W, L, V, x = cat("W"), cat("L"), cat("VTH0"), cat("x")
        B.set_params(W, L, V)
        A = torch.empty(B.nnz, dtype=torch.float64, device=dev)
        b = torch.empty(B.n_rows, dtype=torch.float64, device=dev)
        ms = time_eager(torch, lambda: B.eval_stamp(x, AG0, None, A, b), args.steps, args.warmup)
        B.check()
        log(f"batch 512 region block 256: {ms * 1e3:.1f} us per step ({args.steps} steps)")
        Ab, bb = G.cotangents(B.nnz, B.n_rows, seed=50)
        Ab, bb = torch.from_numpy(Ab).to(dev), torch.from_numpy(bb).to(dev)
        ms_a = time_eager(torch, lambda: B.vjp(x, AG0, Ab, bb), args.steps, args.warmup)
        B.check()
        log(f"batch 512 adjoint: {ms_a * 1e3:.1f} us per step ({ms_a / ms:.2f} x the forward)")
        release(torch, B)
        return
    if args.csweep:
        rows = bench_csweep(torch, CS, G, dev, steps=args.steps)
        print(json.dumps({"sweep": "colour count", "unit": "M devices/s", "launch": "graph replay",
                          "steps": args.steps, "rows": rows}), flush=True)
        return
    khash = kernel_sources_hash()
    circ = G.workload(1)
    log(f"workload: chain 100000 stages, {circ.n_dev} devices")
    counts = algorithmic_counts(circ)
    W, L, V, x = device_tensors(torch, circ, dev)

    variants = {}
    todo = (("persistent", True), ("persistent", False), ("per_kernel", True),
            ("buffered", True), ("region", True), ("atomic", True), ("atomic_wave", True))
    if args.only:
        todo = ((args.variant, True),)
    coop_main = not (args.only and args.ordinary)
    for variant, coop in todo:
        c = CS.prepare(circ, exclude=True)
        c.set_launch(256, -1, coop and coop_main)
        c.set_params(W, L, V)
        A = torch.empty(c.nnz, dtype=torch.float64, device=dev)
        b = torch.empty(c.n_rows, dtype=torch.float64, device=dev)
        steps = args.steps if variant == args.variant and coop else max(10, args.steps // 4)
        ms, g = time_graph(torch, lambda: c.eval_stamp(x, AG0, None, A, b, variant), steps, args.warmup)
        c.check()
        del g
        if variant == args.variant and coop:
            kernel_ms = time_eager(torch, lambda: c.eval_stamp(x, AG0, None, A, b, variant), steps, args.warmup)
            log(f"  {variant} kernel launches back to back: {kernel_ms * 1e3:.2f} us")
            trials = sorted(time_graph(torch, lambda: c.eval_stamp(x, AG0, None, A, b, variant), steps,
                                       args.warmup)[0] for _ in range(5))
            cold_ms = time_cold(torch, lambda: c.eval_stamp(x, AG0, None, A, b, variant), max(10, steps // 4))
            log(f"  {variant} graph replay, median of 5 trials: {trials[2] * 1e3:.2f} us; "
                f"cold (512 MiB flushed before each step): {cold_ms * 1e3:.2f} us")
        name = variant if coop else variant + "_ordinary_launch"
        variants[name] = dict(ms_per_step=round(ms, 5), value=round(circ.n_dev / ms / 1e3, 2),
                              info=c.info(), steps=steps, launch="graph replay")
        if variant == args.variant and coop:
            variants[name]["stream_ms_per_step"] = round(kernel_ms, 5)
            variants[name]["graph_trials_ms"] = [round(t, 5) for t in trials]
            variants[name]["graph_median_of_5_trials_ms"] = round(trials[2], 5)
            variants[name]["cold_ms_per_step"] = round(cold_ms, 5)
            variants[name]["cold_value"] = round(circ.n_dev / cold_ms / 1e3, 2)
        log(f"  {name:28s} {ms * 1e3:9.2f} us/step  {circ.n_dev / ms / 1e3:9.1f} M devices/s")
        release(torch, c)

    main_v = variants[args.variant]
    # a step is one launch sequence of the variant; K steps run either as K replays of
    # a captured graph or as K launches back to back on the stream: the faster counts
    launch = "graph replay" if main_v["ms_per_step"] <= kernel_ms else "stream, back to back"
    ms = min(main_v["ms_per_step"], round(kernel_ms, 5))
    result = {
        "metric": "M devices eval+stamp/s per NR iter (colored vs atomic); batched & fwd+adjoint",
        "value": round(circ.n_dev / ms / 1e3, 2),
        "unit": "M devices/s",
        "n_gpus": 1,
        "steps": main_v["steps"],
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "inverter_chain_100k_stages", "n_dev": circ.n_dev,
                   "n_rows": int(main_v["info"]["n_rows"]), "nnz": int(main_v["info"]["nnz"]),
                   "n_colors": counts["n_colors"], "conflict_rule": "rails_excluded",
                   "variant": args.variant, "ag0": AG0, "launch": launch},
        "roofline": roofline(counts, kernel_ms, traffic_from_profiles(khash, f"{args.variant}_chain100k"),
                             KERNEL_OF.get(args.variant, args.variant)),
        "variants": variants,
        "kernel_sources": khash,
    }

    if not args.no_extras:
        extras = {}
        sram = G.workload(2)
        Ws, Ls, Vs, xs = device_tensors(torch, sram, dev)
        ex = {}
        for variant in ("persistent", "per_kernel", "region", "atomic", "atomic_wave"):
            c = CS.prepare(sram, exclude=True)
            c.set_params(Ws, Ls, Vs)
            A = torch.empty(c.nnz, dtype=torch.float64, device=dev)
            b = torch.empty(c.n_rows, dtype=torch.float64, device=dev)
            step = lambda: c.eval_stamp(xs, AG0, None, A, b, variant)
            msg, _ = time_graph(torch, step, 5, 2)
            mss = time_eager(torch, step, 5, 2)
            msv = min(msg, mss)   # the faster of graph replay and stream launches
            c.check()
            ex[variant] = dict(ms_per_step=round(msv, 4), value=round(sram.n_dev / msv / 1e3, 2),
                               graph_ms_per_step=round(msg, 4), stream_ms_per_step=round(mss, 4))
            log(f"  sram {variant:12s} {msv:8.3f} ms/step {sram.n_dev / msv / 1e3:9.1f} M devices/s")
        extras["sram_256x256"] = dict(n_dev=sram.n_dev, n_colors=c.info()["n_colors"], **ex)
        extras["adder_64bit_28T"] = bench_adder(torch, CS, G, dev)
        extras["batch_512"] = bench_batch(torch, CS, G, dev)
        extras["adjoint"] = bench_adjoint(torch, CS, G, dev)
        extras["junction_level"] = bench_junction_level(torch, CS, G, dev)
        extras["newton"] = bench_newton(torch, CS, G, dev)
        result["extras"] = extras

    # the paper's own CPU figures, for context only (another machine, full BSIM 4.82):
    # FET evaluations per second derived from its Device-Eval times (1792 FETs x NR
    # iterations / seconds) on a 64-core Threadripper PRO 5995WX, and its best speedup
    result["paper_context"] = {
        "hardware": "AMD Ryzen Threadripper PRO 5995WX, 64 cores, C++/OpenMP, BSIM 4.82",
        "colorfused_fet_evals_per_s_M": {"adder_base_C896": 0.707, "adder_R14_C64": 7.74, "adder_R89_C1": 24.8},
        "loadomp_fet_evals_per_s_M": 7.42, "ngspice_fet_evals_per_s_M": 4.93,
        "colorfused_best_speedup_vs_1_thread": 45,
    }
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(circ)
        log(f"  cpu oracle: {result['cpu_baseline']['value']} M devices/s")
    print(json.dumps(result), flush=True)
    # every captured graph and handle is gone before the interpreter exits
    import gc
    gc.collect()
    torch.cuda.synchronize()
    CS._close_all()


if __name__ == "__main__":
    main()
