"""Benchmark: station-unfolds/s of the FP32 batched path, with the FP64 plain
path on the same GPU, the HBM roofline of the dominant kernel and the CPU
oracle as a reported baseline.

Workloads (synthetic, AERA-shaped; see paper_1507_07733_amd/synth.py):
* batched FP32 (the value): 256 events, stations uniform in 3..124, traces of
  2048 or 4096 float32 samples (equal odds), 16 x 16 candidate directions
  per event, complex64 pattern table on the 0.5 MHz / 1 deg grid, FP32
  compute with the FP64 determinant fallback, one batched plan.
* FP64 plain: one event of 124 stations x 4096 float64 samples, 32 x 64
  directions, complex128 table on the 1 MHz / 5 deg grid,
  au_unfold_direction_scan in FP64.

A station-unfold is one (event, direction, station) producing E_theta and
E_phi traces.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM bytes per launch of the dominant kernel on this workload: rocprofv3 FETCH_SIZE x 2.000 +
# WRITE_SIZE x 1.000 (copy-probe calibration), keyed by kernel and launch size.
PROFILED_TRAFFIC_SOURCE = "profiles/k_unfold_fp32_batched_256events.md"
PROFILED_TRAFFIC_BYTES = {
    ("k_unfold<float, 4096, 8, 8, 4, false, false, true>", 2047488): (1180268 + 65522388) * 1024,
}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_batched_workload(n_events=256, seed_cfg=2):
    from paper_1507_07733_amd import synth
    dirs = synth.direction_grid(16, 16)
    ev = synth.event_mix(n_events, cfg=seed_cfg, dirs=dirs)
    specs = [(e.n_stations, e.n_samples, dirs) for e in ev]
    return specs


def gen_traces(specs, offsets, total, seed_cfg=2):
    from paper_1507_07733_amd import synth
    volt = np.empty(total, dtype=np.float32)

    def one(e):
        s, n, _ = specs[e]
        v = synth.traces(s, n, cfg=seed_cfg, event=e, dtype=np.float32)
        volt[offsets[e]:offsets[e] + v.size] = v.ravel()
        return e

    with cf.ThreadPoolExecutor(8) as ex:
        list(ex.map(one, range(len(specs))))
    return volt


def cgroup_cpu_quota():
    """CPUs granted by the cgroup's CPU quota (None if unlimited or unknown)."""
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, p = f.read().split()[:2]
        if q != "max":
            return float(q) / float(p)
    except (OSError, ValueError):
        pass
    try:
        with open("/sys/fs/cgroup/cpu/cpu.cfs_quota_us") as f:
            q = float(f.read())
        with open("/sys/fs/cgroup/cpu/cpu.cfs_period_us") as f:
            p = float(f.read())
        if q > 0:
            return q / p
    except (OSError, ValueError):
        pass
    return None


def cpu_threads():
    """Every host core this process may use: its CPU affinity, bounded by the cgroup's CPU quota
    (a GPU machine grants each job a share of its cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:
        n = os.cpu_count() or 1
    q = cgroup_cpu_quota()
    if q is not None:
        n = min(n, max(1, int(q)))
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(grid, table_c64, specs, plan, volt_host, budget_s=12.0):
    """Oracle throughput on a bounded sample of the batched workload.

    Random (event, direction, station) units of the same workload, in chunks
    of 16 units, run on a thread pool over the host cores (the oracle is C
    called through ctypes, which releases the GIL) until budget_s of wall
    time has passed.
    """
    from oracle import oracle as O
    from paper_1507_07733_amd import synth
    t128 = np.asarray(table_c64).astype(np.complex128)
    threads = cpu_threads()

    def task(i):
        e = int((i * 7919) % len(specs))
        s, n, dirs = specs[e]
        o = plan.volt_offsets[e]
        v = volt_host[o:o + s * 2 * n].reshape(s, 2, n).astype(np.float64)
        r = np.random.default_rng(i)
        units = np.stack([r.integers(len(dirs), size=16), r.integers(s, size=16)], axis=1)
        O.unfold(grid, t128, v, dirs, synth.FS_HZ, synth.BAND_LO_HZ, synth.BAND_HI_HZ, units=units)
        return 16, n

    O.lib()
    done = 0
    n_by = {2048: 0, 4096: 0}
    t0 = time.perf_counter()
    i = 0
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = set()
        while True:
            while len(futs) < 2 * threads and time.perf_counter() - t0 < budget_s:
                futs.add(ex.submit(task, i))
                i += 1
            if not futs:
                break
            fin, futs = cf.wait(futs, return_when=cf.FIRST_COMPLETED)
            for f in fin:
                u, n = f.result()
                done += u
                n_by[n] = n_by.get(n, 0) + u
    wall = time.perf_counter() - t0
    # the same tasks on one thread, for the per-core rate
    done1 = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < budget_s / 4:
        done1 += task(i)[0]
        i += 1
    wall1 = time.perf_counter() - t1
    return {"value": done / wall, "unit": "station-unfolds/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cgroup_cpus": cgroup_cpu_quota(),
            "cpu_model": cpu_model(),
            "sample": "%d random (event, direction, station) units of the batched workload "
                      "(%d at N=2048, %d at N=4096), FP64 on the float32 inputs, %.1f s wall on %d threads"
                      % (done, n_by.get(2048, 0), n_by.get(4096, 0), wall, threads),
            "single_thread_value": done1 / wall1}


def parity_sample(grid, table_c64, specs, plan, volt_host, efield, n_units=8):
    """Max per-trace error of a few sampled units against the oracle."""
    from oracle import oracle as O
    from paper_1507_07733_amd import synth
    t128 = np.asarray(table_c64).astype(np.complex128)
    worst = 0.0
    r = np.random.default_rng(99)
    for _ in range(n_units):
        e = int(r.integers(len(specs)))
        s, n, dirs = specs[e]
        d, st = int(r.integers(len(dirs))), int(r.integers(s))
        o = plan.volt_offsets[e]
        v = volt_host[o:o + s * 2 * n].reshape(s, 2, n).astype(np.float64)
        ref, _, _ = O.unfold(grid, t128, v, dirs, synth.FS_HZ, synth.BAND_LO_HZ, synth.BAND_HI_HZ,
                             units=[[d, st]])
        got = plan.event_output(efield, e)[d, st].cpu().numpy().astype(np.float64)
        err = np.max(np.abs(got - ref[0]), axis=-1) / np.max(np.abs(ref[0]), axis=-1)
        worst = max(worst, float(err.max()))
    return worst


KAPPA_EDGES = (1.0, 3.0, 10.0, 30.0, 100.0, 1e3, float("inf"))
SHARE_EDGES = (0.0, 0.01, 0.1, 1.0 + 1e-12)


def fp32_error_report(api, plan, specs, efield, tab64, volt, dev):
    """FP32 batched output vs the FP64 path for every output trace.

    Per event the FP64 direction scan (complex128 table, same float32
    traces) runs on the device; per trace r = max|E32 - E64| / max|E64|.
    Traces are bucketed by kappa = max over in-band bins of ||H||_F^2/|det|
    of their direction (from au_pattern_response in FP64)."""
    import torch
    buckets = {i: [] for i in range(len(KAPPA_EDGES) - 1)}
    sbuckets = {i: [] for i in range(len(KAPPA_EDGES) - 1)}
    shbuckets = {i: [] for i in range(len(SHARE_EDGES) - 1)}
    worst = worst_s = 0.0
    n_tr = 0
    for e, (s, n, dirs) in enumerate(specs):
        ev64 = api.make_event(s, n, prec=api.AU_PREC_FP64, trace_dtype=api.AU_F32)
        o = int(plan.volt_offsets[e])
        v = volt[o:o + s * 2 * n].view(s, 2, n)
        e64 = api.unfold_direction_scan(tab64, ev64, v, dirs)
        e32 = plan.event_output(efield, e)
        ref = e64.abs().amax(dim=-1)                                   # [D][S][2]
        dif = (e32.double() - e64).abs().amax(dim=-1)
        err = dif / torch.where(ref > 0, ref, torch.ones_like(ref))
        ref_s = ref.amax(dim=-1)                                       # the station's E-field trace
        err_s = dif.amax(dim=-1) / torch.where(ref_s > 0, ref_s, torch.ones_like(ref_s))
        h = api.pattern_response(tab64, ev64, dirs)              # [D][nb][2][2] complex128
        det = h[:, :, 0, 0] * h[:, :, 1, 1] - h[:, :, 0, 1] * h[:, :, 1, 0]
        fro2 = (h.abs() ** 2).sum(dim=(-1, -2))
        kappa = (fro2 / det.abs()).amax(dim=-1)                  # [D]
        kb = torch.bucketize(kappa, torch.tensor(KAPPA_EDGES[1:-1], dtype=kappa.dtype, device=kappa.device))
        err_d = err.reshape(len(dirs), -1).cpu().numpy()
        err_sd = err_s.reshape(len(dirs), -1).cpu().numpy()
        kb = kb.cpu().numpy()
        for di in range(len(dirs)):
            buckets[int(kb[di])].append(err_d[di])
            sbuckets[int(kb[di])].append(err_sd[di])
        share = (ref / torch.where(ref_s > 0, ref_s, torch.ones_like(ref_s)).unsqueeze(-1)).reshape(-1)
        sb = torch.bucketize(share, torch.tensor(SHARE_EDGES[1:-1], dtype=share.dtype, device=share.device))
        ef, sb = err.reshape(-1).cpu().numpy(), sb.cpu().numpy()
        for i in range(len(SHARE_EDGES) - 1):
            shbuckets[i].append(ef[sb == i])
        worst = max(worst, float(err.max()))
        worst_s = max(worst_s, float(err_s.max()))
        n_tr += err.numel()
        del e64
    out = []
    for i, lst in buckets.items():
        if not lst:
            continue
        a = np.concatenate(lst)
        b = np.concatenate(sbuckets[i])
        out.append({"kappa": [KAPPA_EDGES[i], KAPPA_EDGES[i + 1]], "traces": int(a.size),
                    "max": float(a.max()), "p99": float(np.percentile(a, 99)), "median": float(np.median(a)),
                    "max_station": float(b.max())})
    by_share = []
    for i, lst in shbuckets.items():
        a = np.concatenate(lst) if lst else np.zeros(0)
        if not a.size:
            continue
        by_share.append({"share": [SHARE_EDGES[i], SHARE_EDGES[i + 1]], "traces": int(a.size),
                         "max": float(a.max()), "p99": float(np.percentile(a, 99)), "median": float(np.median(a)),
                         "over_1e-5": int(np.sum(a > 1e-5))})
    return {"traces": n_tr, "max": worst, "max_station": worst_s, "by_kappa": out, "by_component_share": by_share,
            "reference": "FP64 direction scan on the same float32 traces (complex128 table)",
            "normalisation": "max/p99/median: per component trace, max|E32-E64| / max|E64| of that component; "
                             "max_station: per station, over both components, divided by the larger peak; "
                             "by_component_share: per component, bucketed by the component's peak over the "
                             "station's peak (the FP32 rule: per station, and per component from share 0.1)"}


# FP32 vector FMA rate without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


# Dynamic VALU instructions (wave-instructions) per station-unfold of the dominant kernel, from the
# committed SQ_INSTS_VALU profile of the same build and workload, keyed like the traffic.
PROFILED_VALU_INSTR = {
    ("k_unfold<float, 4096, 8, 8, 4, false, false, true>", 2047488): 2462.0,
}
# wave64 VALU issue without packed FP32: one instruction per SIMD every 4 cycles, 1024 SIMDs at 2.4 GHz
VALU_ISSUE_PEAK_GINSTR = 256 * 4 * 2.4e9 / 4 / 1e9


def valu_issue_view(cls):
    """The dominant launch against the VALU issue rate: profiled instructions per station-unfold x the
    launch's station-unfolds over its time, against the nominal-clock issue limit (the chip runs this
    kernel at 1.7-1.8 GHz, so the limit at the sustained clock is about 0.72 of the nominal one)."""
    per = PROFILED_VALU_INSTR.get((cls["kernel"], cls["station_unfolds"]))
    if per is None:
        return None
    achieved = per * cls["station_unfolds"] / (cls["unfold_ms"] / 1e3) / 1e9
    return {"bound": "alu", "achieved": round(achieved, 1), "peak": round(VALU_ISSUE_PEAK_GINSTR, 1),
            "unit": "G wave-instructions/s", "frac": round(achieved / VALU_ISSUE_PEAK_GINSTR, 4),
            "instructions_per_unit": per, "source": PROFILED_TRAFFIC_SOURCE}


def alu_view(cls):
    """The dominant launch against the vector ALU: algorithmic flops per station-unfold (inverse
    complex FFT at 5 N log2 N, plus 4 complex multiply-adds per in-band bin) over the launch time."""
    n = cls["n_samples"]
    nb = n // 4                                   # 30-80 MHz of 0-100 MHz at 200 MHz: a quarter of the bins
    flops = 5 * n * int(np.log2(n)) + nb * 28
    achieved = cls["station_unfolds"] * flops / (cls["unfold_ms"] / 1e3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": round(FP32_VALU_PEAK_TFLOPS, 1),
            "unit": "TFLOP/s", "frac": round(achieved / FP32_VALU_PEAK_TFLOPS, 4),
            "flops_per_unit": flops, "convention": "5 N log2 N per complex FFT + 28 flops per in-band bin"}


def settle(fn, seconds=0.25):
    """Call fn back to back for about `seconds`: an idle GPU lowers its clocks and needs tens of
    milliseconds of load to return to its steady state (the 124-station FP64 scan takes 4.3-4.6 ms
    per call after a 50 ms pause, 3.5-3.6 ms back to back), so a timed section starts after this."""
    import torch
    t0 = time.perf_counter()
    while True:
        fn()
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            return


def envelope_scan_rate(api, tab, ev, volt, dirs, work, reps, stream):
    """Station-unfolds/s of au_unfold_envelope_scan (peaks and their samples only, no traces)."""
    import torch
    settle(lambda: api.unfold_envelope_scan(tab, ev, volt, dirs, work=work))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        api.unfold_envelope_scan(tab, ev, volt, dirs, work=work)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    su = len(dirs) * ev.n_stations
    n = ev.n_samples
    # 2 complex inverse FFTs per station-unfold at the 5 N log2 N convention
    flops = su * 2 * 5 * n * int(np.log2(n))
    return {"value": su / (ms / 1e3), "unit": "station-unfolds/s", "ms_per_call": ms, "station_unfolds": su,
            "fft_GFLOPs_5NlogN": flops / (ms / 1e3) / 1e9}


def reconstruction_latency(api, synth, tab64, tab32, dev, n_events=8, n_st=124, n=4096, max_iter=8):
    """Wall time per event of the device reconstruction loop on plane-wave events
    (124 stations on the 6 km^2 hexagonal layout, directions spread over the sky)."""
    import torch
    pos = synth.station_positions(n_st)
    r = synth.rng(5, synth.STREAM_EVENTS)
    truth = np.stack([r.uniform(5.0, 65.0, n_events), r.uniform(0.0, 360.0, n_events)], 1)
    out = {}
    for name, tab, prec, tin, dt in (("fp64", tab64, api.AU_PREC_FP64, api.AU_F64, np.float64),
                                     ("fp32", tab32, api.AU_PREC_FP32, api.AU_F32, np.float32)):
        ev = api.make_event(n_st, n, prec=prec, trace_dtype=tin)
        work = torch.empty(api.reconstruct_workspace_bytes(tab, ev, max_iter), dtype=torch.uint8, device=dev)
        vols = [torch.from_numpy(synth.plane_wave_traces(pos, n, z, a, cfg=5, event=i, dtype=dt)[0]).to(dev)
                for i, (z, a) in enumerate(truth)]
        api.reconstruct(tab, ev, vols[0], pos, max_iter=max_iter, work=work)
        torch.cuda.synchronize()
        passes, conv, err = [], 0, []
        t0 = time.perf_counter()
        for i, v in enumerate(vols):
            rec = api.reconstruct(tab, ev, v, pos, max_iter=max_iter, work=work)
            passes.append(len(rec.dirs))
            conv += rec.converged
            z, a = np.radians(rec.direction)
            zt, at = np.radians(truth[i])
            cosang = np.sin(z) * np.sin(zt) * np.cos(a - at) + np.cos(z) * np.cos(zt)
            err.append(np.degrees(np.arccos(min(1.0, cosang))))
        ms = (time.perf_counter() - t0) * 1e3 / n_events
        out[name] = {"ms_per_event": ms, "mean_passes": float(np.mean(passes)), "converged": int(conv),
                     "events": n_events, "max_angle_err_deg": float(np.max(err))}
        # the same events many times over in one batched call (inputs shared round-robin)
        n_batch = 512
        flat = torch.cat([v.reshape(-1) for v in vols])
        vsz = n_st * 2 * n
        offs = [(i % n_events) * vsz for i in range(n_batch)]
        allpos = np.tile(pos, (n_batch, 1))
        api.reconstruct_batch(tab, ev, flat, [n_st] * n_batch, offs, allpos, max_iter=max_iter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = api.reconstruct_batch(tab, ev, flat, [n_st] * n_batch, offs, allpos, max_iter=max_iter)
        ms_b = (time.perf_counter() - t0) * 1e3
        out[name]["batch"] = {"events": n_batch, "ms": ms_b, "events_per_s": n_batch / (ms_b / 1e3),
                              "converged": int(sum(r.converged == 1 for r in res))}
        del vols, work, flat
    out["workload"] = "%d plane-wave events, %d stations (hexagonal, 6 km^2) x %d samples, max %d passes" % (
        n_events, n_st, n, max_iter)
    return out


def direction_fit_latency(api, synth, tab64, dev, n_events=4, n_st=124, n=4096, levels=4, k=5, fp32=False):
    """Wall time per event of the device direction fit: 32 x 64 coarse candidates (the FP64 scan's grid)
    plus `levels` 5 x 5 refinements, on plane-wave events."""
    import torch
    pos = synth.station_positions(n_st)
    r = synth.rng(6, synth.STREAM_EVENTS)
    truth = np.stack([r.uniform(5.0, 65.0, n_events), r.uniform(0.0, 360.0, n_events)], 1)
    coarse = synth.direction_grid(32, 64)
    if fp32:
        ev = api.make_event(n_st, n, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32)
    else:
        ev = api.make_event(n_st, n)
    dt = np.float32 if fp32 else np.float64
    work = torch.empty(api.direction_fit_workspace_bytes(tab64, ev, len(coarse), levels, k), dtype=torch.uint8,
                       device=dev)
    vols = [torch.from_numpy(synth.plane_wave_traces(pos, n, z, a, cfg=6, event=i, dtype=dt)[0]).to(dev)
            for i, (z, a) in enumerate(truth)]
    step = (90.0 / 32, 360.0 / 64)
    api.direction_fit(tab64, ev, vols[0], pos, coarse, levels=levels, k=k, step=step, work=work)
    torch.cuda.synchronize()
    err = []
    t0 = time.perf_counter()
    for i, v in enumerate(vols):
        fit = api.direction_fit(tab64, ev, v, pos, coarse, levels=levels, k=k, step=step, work=work)
        z, a = np.radians(fit["result"])
        zt, at = np.radians(truth[i])
        cosang = np.sin(z) * np.sin(zt) * np.cos(a - at) + np.cos(z) * np.cos(zt)
        err.append(np.degrees(np.arccos(min(1.0, cosang))))
    ms = (time.perf_counter() - t0) * 1e3 / n_events
    su = (len(coarse) + levels * k * k) * n_st
    return {"ms_per_event": ms, "station_unfolds_per_event": su, "station_unfolds_per_s": su / (ms / 1e3),
            "max_angle_err_deg": float(np.max(err)), "events": n_events,
            "workload": "%s, %d plane-wave events, %d stations x %d samples, 32x64 candidates + %d levels of %dx%d"
                        % ("FP32" if fp32 else "FP64", n_events, n_st, n, levels, k, k)}


def large_batch_rate(api, synth, tab32, grid, table_c64, dev, n_events=10000, n_st=124, n=4096, ring=100, kept=100,
                     steps=3, sample_units=2):
    """The large-batch workload (10 000 events x 124 stations x 4096 float32 samples x 4 x 4 directions)
    through the batched plan captured in a hipGraph.  All 10 000 input events are distinct (40.6 GB,
    generated on the device by the counter-based stream of synth.stream_traces).  The 650 GB of output
    exceed HBM: the first `kept` events own their output slots, the others write into a ring of `ring`
    slots after them (overlapping writes, for throughput).  The FP32 error against the FP64 oracle is
    measured on a 1 % sample: `sample_units` (direction, station) units of each kept event, the oracle
    fed the same traces regenerated on the host."""
    import torch
    from oracle import oracle as O
    dirs = synth.direction_grid(4, 4)
    specs = [(n_st, n, dirs)] * n_events
    vsz = n_st * 2 * n
    esz = len(dirs) * n_st * 2 * n
    volt_off = np.arange(n_events, dtype=np.int64) * vsz
    idx = np.arange(n_events)
    eff = np.where(idx < kept, idx, kept + (idx % ring)).astype(np.int64) * esz
    plan = api.Plan(tab32, specs, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32, flags=7 | api.AU_PLAN_FUSED,
                    volt_offsets=volt_off, efield_offsets=eff)
    t0 = time.perf_counter()
    dv = torch.empty(n_events * vsz, dtype=torch.float32, device=dev)
    chunk = 500
    for e0 in range(0, n_events, chunk):
        k = min(chunk, n_events - e0)
        synth.device_stream_traces(dv[e0 * vsz:(e0 + k) * vsz], e0, k, n_st, n)
    gen_s = time.perf_counter() - t0
    out = torch.empty(plan.efield_elems, dtype=torch.float32, device=dev)
    plan.run(dv, out)
    torch.cuda.synchronize()
    e0_, e1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0_.record()
    for _ in range(steps):
        plan.run(dv, out)
    e1_.record()
    torch.cuda.synchronize()
    ms = e0_.elapsed_time(e1_) / steps
    su = plan.station_unfolds
    # the same workload with separate spectrum and unfold stages, for comparison
    plan_sep = api.Plan(tab32, specs, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32, flags=7, volt_offsets=volt_off,
                        efield_offsets=eff)
    plan_sep.run(dv, out)
    torch.cuda.synchronize()
    e0_.record()
    for _ in range(steps):
        plan_sep.run(dv, out)
    e1_.record()
    torch.cuda.synchronize()
    ms_sep = e0_.elapsed_time(e1_) / steps
    del plan_sep
    plan.run(dv, out)                    # the kept slots hold the fused plan's output again
    torch.cuda.synchronize()
    # 1 % sample against the oracle (the kept events' own slots hold their last run's output)
    r = np.random.default_rng(41)
    t128 = np.asarray(table_c64).astype(np.complex128)
    worst_s = worst_c = 0.0
    n_units = 0
    for e in range(kept):
        for _ in range(sample_units):
            d, st = int(r.integers(len(dirs))), int(r.integers(n_st))
            v1 = synth.stream_traces([e], n_st, n, stations=[st])[0]
            ref, _, _ = O.unfold(grid, t128, v1.astype(np.float64), dirs, synth.FS_HZ, synth.BAND_LO_HZ,
                                 synth.BAND_HI_HZ, units=[[d, 0]])
            got = plan.event_output(out, e)[d, st].cpu().numpy().astype(np.float64)
            pk = np.max(np.abs(ref[0]), axis=-1)
            err = np.max(np.abs(got - ref[0]), axis=-1)
            worst_s = max(worst_s, float(err.max() / pk.max()))
            strong = pk >= 0.1 * pk.max()
            worst_c = max(worst_c, float(np.max(err[strong] / pk[strong])))
            n_units += 1
    res = {"value": su / (ms / 1e3), "unit": "station-unfolds/s", "ms_per_step": ms, "station_unfolds": su,
           "output_GBs": su * 2 * n * 4 / (ms / 1e3) / 1e9,
           "input_GB": n_events * vsz * 4 / 1e9, "generation_s": gen_s,
           "separate_stages_ms_per_step": ms_sep,
           "fp32_error_vs_oracle": {"units": n_units, "events": kept, "max_station": worst_s,
                                    "max_strong_component": worst_c,
                                    "sample": "%d random (direction, station) units of each of the %d events that "
                                              "own their output slots (1 %% of the events)" % (sample_units, kept)},
           "workload": "%d distinct events x %d stations x %d float32 samples (generated on the device) x 16 "
                       "directions, complex64 table, hipGraph, fused spectrum + unfold; outputs of %d events "
                       "kept, the rest recycled through a %d-event ring" % (n_events, n_st, n, kept, ring)}
    del out, dv, plan
    torch.cuda.empty_cache()
    return res


def single_event_latency(api, synth, dev, calls=300, warm=20):
    """The plain FP64 single-event call (10 stations x 2 channels x 2048 float64 samples, one
    direction (40, 120) deg, complex128 table 1 MHz / 5 deg): wall time per call including the wait
    for its completion (the latency a caller sees), and the device time of its launches (HIP events
    on the call's stream)."""
    import torch
    g = synth.GRID_COARSE
    tb = api.Table(g, synth.pattern_table(g, cfg=0))
    v = torch.from_numpy(synth.traces(10, 2048, cfg=0, event=0)).to(dev)
    ev = api.make_event(10, 2048, prec=api.AU_PREC_FP64, trace_dtype=api.AU_F64)
    out = torch.empty((10, 2, 2048), dtype=torch.float64, device=dev)
    work = torch.empty(api.workspace_bytes(tb, ev, 1), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    wall, gpu = [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i in range(warm + calls):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        api.unfold_event(tb, ev, v, 40.0, 120.0, out=out, work=work)
        e1.record(stream)
        e1.synchronize()
        t1 = time.perf_counter()
        if i >= warm:
            wall.append((t1 - t0) * 1e6)
            gpu.append(e0.elapsed_time(e1) * 1e3)
    wall, gpu = np.array(wall), np.array(gpu)
    return {"us_per_call_median": float(np.median(wall)), "us_per_call_min": float(wall.min()),
            "device_us_median": float(np.median(gpu)), "device_us_min": float(gpu.min()), "calls": calls,
            "workload": "plain FP64 au_unfold_event: 10 stations x 2 x 2048 float64 samples at 200 MHz, one "
                        "direction (40, 120) deg, complex128 table 1 MHz/5 deg; wall time per call until complete"}


def serve_stream(api, sv, vols, dirs, arrivals, warm_s):
    """Submit each event at its scheduled arrival (open loop: a producer thread spins to the arrival
    time, so a slow server never delays later arrivals), wait for every result in order, and return
    latency statistics over the events arriving after warm_s."""
    import threading
    n_ev = len(arrivals)
    pool = len(vols)
    tickets = [None] * n_ev
    t_start = sv.now() + 0.2
    rejected = [0]
    failure = []

    def producer():
        try:
            for i, a in enumerate(arrivals):
                target = t_start + a
                while sv.now() < target:
                    pass
                while True:
                    try:
                        tickets[i] = sv.submit(vols[i % pool], dirs, t_arrival=target)
                        break
                    except api.AuError as e:
                        if e.status != api.AU_EAGAIN:
                            raise
                        rejected[0] += 1
                        time.sleep(1e-4)
        except Exception as e:  # reported by the consumer below
            failure.append(e)

    th = threading.Thread(target=producer)
    th.start()
    lat, batch, done_t, parts, units = [], [], [], [], 0
    for i in range(n_ev):
        while tickets[i] is None:
            if failure:
                th.join()
                raise failure[0]
            time.sleep(2e-5)
        res = sv.wait(tickets[i], timeout_s=120)
        if arrivals[i] >= warm_s:
            lat.append(res.t_complete - res.t_arrival)
            parts.append((res.t_submit - res.t_arrival, res.t_admit - res.t_submit, res.t_launch - res.t_admit,
                          res.t_complete - res.t_launch))
            batch.append(res.batch_events)
            done_t.append(res.t_complete)
            units += res.n_stations * res.n_dirs
        sv.release(tickets[i])
    th.join()
    st = sv.stats()
    lat = np.array(lat) * 1e3
    parts = np.array(parts) * 1e3
    span = max(done_t) - (t_start + warm_s)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "events": len(lat),
            "events_per_s": len(lat) / span, "station_unfolds_per_s": units / span,
            "mean_batch_events": float(np.mean(batch)), "max_batch_events": int(np.max(batch)),
            "submit_retries": rejected[0], "arena_peak_GB": st["arena_peak"] / 1e9,
            "median_ms": {"arrival_to_submit_return": float(np.median(parts[:, 0] + parts[:, 1])),
                          "submit_to_admit": float(np.median(parts[:, 1])),
                          "admit_to_launch": float(np.median(parts[:, 2])),
                          "launch_to_complete": float(np.median(parts[:, 3]))}}


def serving_benchmark(api, synth, tab32, tab64, rate_hz=2000.0, duration_s=3.0, warm_s=0.5,
                      plain_s=1.5, pool=48, burst_rate_hz=40000.0, burst_s=0.5):
    """Open-loop Poisson stream of events (stations U{3..124}, 2048 float32
    samples, 8x8 directions) served by the continuous-batching server, and the
    same stream by a plain FP64 per-event loop.  Latency = completion time -
    scheduled arrival time (no coordinated omission); the first warm_s
    seconds are discarded.  Traces are submitted from pinned host memory, as
    the plain loop copies them.  A second, saturated load point offers
    burst_rate_hz (beyond what the device serves) with a 1 ms batching tick,
    so events are grouped into shared launches."""
    import torch
    r = synth.rng(3, synth.STREAM_EVENTS)
    sizes = r.integers(3, 125, size=pool)
    vols = [synth.traces(int(sz), 2048, cfg=3, event=i, dtype=np.float32) for i, sz in enumerate(sizes)]
    vols_pinned = [torch.from_numpy(v).pin_memory() for v in vols]
    dirs = synth.direction_grid(8, 8)
    arrivals = synth.poisson_arrivals(rate_hz, duration_s, cfg=3)
    sv = api.Server(tab32, hbm_budget_bytes=48 << 30, staging_bytes=4 << 30, max_inflight=256,
                    n_streams=4, max_batch_events=16, tick_s=0.0)
    try:
        served = serve_stream(api, sv, vols_pinned, dirs, arrivals, warm_s)
    finally:
        sv.close()
    served.update({"offered_events_per_s": rate_hz, "tick_s": 0.0,
                   "workload": "Poisson %.0f events/s for %.1f s (first %.1f s discarded), stations U{3..124}, "
                               "2048 float32 samples, 8x8 directions, FP32 server, 4 streams, traces submitted "
                               "from pinned host memory" % (rate_hz, duration_s, warm_s)})
    # saturated point: more offered than served, micro-batches gathered over a 1 ms tick
    arr_b = np.sort(synth.rng(3, synth.STREAM_ARRIVALS, 1).uniform(0.0, burst_s, int(burst_rate_hz * burst_s)))
    sv = api.Server(tab32, hbm_budget_bytes=48 << 30, staging_bytes=2 << 30, max_inflight=512,
                    n_streams=4, max_batch_events=16, tick_s=1e-3)
    try:
        sat = serve_stream(api, sv, vols_pinned, dirs, arr_b, 0.1)
    finally:
        sv.close()
    sat.update({"offered_events_per_s": burst_rate_hz, "tick_s": 1e-3,
                "workload": "uniform arrivals at %.0f events/s for %.1f s (first 0.1 s discarded), same events, "
                            "max 16 events per batch, 1 ms tick" % (burst_rate_hz, burst_s)})
    served["saturated"] = sat

    # plain FP64 per-event loop on the same arrival stream
    dev = torch.device("cuda:0")
    smax = int(sizes.max())
    out_flat = torch.empty(len(dirs) * smax * 2 * 2048, dtype=torch.float64, device=dev)
    ev_max = api.make_event(smax, 2048, prec=api.AU_PREC_FP64, trace_dtype=api.AU_F64)
    work = torch.empty(api.workspace_bytes(tab64, ev_max, len(dirs)), dtype=torch.uint8, device=dev)
    vols64 = [torch.from_numpy(v.astype(np.float64)).pin_memory() for v in vols]
    dvol = torch.empty((smax, 2, 2048), dtype=torch.float64, device=dev)
    sel = arrivals[arrivals < plain_s]
    lat2 = []
    t0 = time.perf_counter() + 0.1
    for i, a in enumerate(sel):
        target = t0 + a
        while time.perf_counter() < target:
            pass
        v = vols64[i % pool]
        s = v.shape[0]
        dv = dvol[:s]
        dv.copy_(v)
        ev = api.make_event(s, 2048, prec=api.AU_PREC_FP64, trace_dtype=api.AU_F64)
        o = out_flat[: len(dirs) * s * 2 * 2048].view(len(dirs), s, 2, 2048)
        api.unfold_direction_scan(tab64, ev, dv, dirs, out=o, work=work)
        torch.cuda.synchronize()
        if a >= warm_s:
            lat2.append(time.perf_counter() - target)
    lat2 = np.array(lat2) * 1e3
    plain = {"p50_ms": float(np.percentile(lat2, 50)), "p99_ms": float(np.percentile(lat2, 99)),
             "events": len(lat2),
             "workload": "same arrivals (first %.1f s), one au_unfold_direction_scan FP64 call per event "
                         "after its host-to-device copy, synchronised" % plain_s}
    served["plain_fp64_loop"] = plain
    return served


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--flags", type=int, default=6, help="plan flags: 1 graph, 2 persistent, 4 XCD placement")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-fp32-error", action="store_true", help="skip the FP32-vs-FP64 error pass over every output")
    ap.add_argument("--no-large-batch", action="store_true", help="skip the 10 000-event large batch")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (library defaults or --variant-*)")
    ap.add_argument("--variant-fp32", default="", help="pin FP32 unfold variants: V (every N >= 1024) or N=V,N=V")
    ap.add_argument("--variant-fp64", default="", help="pin FP64 unfold variants: V (every N >= 1024) or N=V,N=V")
    ap.add_argument("--probe-gib", type=float, default=4.0, help="size of the HBM copy probe")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(events are independent: a multi-GPU run would give each GPU its own events "
              "and its own copy of the pattern table)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1507_07733_amd import api, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    for prec, spec in ((api.AU_PREC_FP32, args.variant_fp32), (api.AU_PREC_FP64, args.variant_fp64)):
        for item in filter(None, spec.split(",")):
            if "=" in item:
                n, v = item.split("=")
                api.set_unfold_variant(prec, int(n), int(v))
            else:
                for n in (1024, 2048, 4096):
                    api.set_unfold_variant(prec, n, int(item))

    # ---------------- HBM copy probe ---------------------------------------
    nbytes = int(args.probe_gib * (1 << 30)) // 16 * 16
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    api.hbm_copy(dst, src, nbytes)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    ev0.record(stream)
    for _ in range(reps):
        api.hbm_copy(dst, src, nbytes)
    ev1.record(stream)
    torch.cuda.synchronize()
    copy_ms = ev0.elapsed_time(ev1) / reps
    copy_gbs = 2 * nbytes / (copy_ms / 1e3) / 1e9
    log("hbm copy probe: %.0f MiB in %.3f ms -> %.0f GB/s (read + write)" % (nbytes / 2**20, copy_ms, copy_gbs))
    del src, dst
    torch.cuda.empty_cache()

    # ---------------- batched FP32 workload -------------------------------
    t0 = time.perf_counter()
    grid = synth.GRID_FINE
    table = synth.pattern_table(grid, cfg=2).astype(np.complex64)
    tab = api.Table(grid, table)
    specs = build_batched_workload(args.events)
    tuned = {}
    flags = args.flags & ~api.AU_PLAN_GRAPH      # stage timing needs eager launches
    plan = api.Plan(tab, specs, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32, flags=flags)
    volt_host = gen_traces(specs, plan.volt_offsets, plan.volt_elems)
    volt = torch.from_numpy(volt_host).to(dev)
    efield = torch.empty(plan.efield_elems, dtype=torch.float32, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    log("batched workload ready: %d events, %d station-unfolds, %.1f GB out, setup %.1f s"
        % (len(specs), plan.station_unfolds, plan.efield_elems * 4 / 1e9, time.perf_counter() - t0))
    if not args.no_tune and not args.variant_fp32:
        # every unfold variant timed inside this plan; the graph plan below takes the same choice
        for n, best, ms in plan.autotune(volt, efield, reps=3):
            api.set_unfold_variant(api.AU_PREC_FP32, n, best)
            tuned["fp32_N%d" % n] = {"variant": best, "shape": api.unfold_variants()[best],
                                     "unfold_ms": [round(m, 4) for m in ms]}
            log("in-plan autotune fp32 N=%d: variant %d %s" % (n, best, api.unfold_variants()[best]))

    for _ in range(args.warmup):
        plan.run(volt, efield, counts)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # eager launches, back to back
    ev0.record(stream)
    for _ in range(args.steps):
        plan.run(volt, efield, counts)
    ev1.record(stream)
    torch.cuda.synchronize()
    eager_ms = ev0.elapsed_time(ev1) / args.steps
    log("batched fp32 eager: %.3f ms/step" % eager_ms)
    # stage timing (HIP events between the launches, one host wait per run) for the roofline
    plan.set_timing(True)
    for _ in range(max(3, args.steps // 3)):
        plan.run(volt, efield, counts)
    torch.cuda.synchronize()
    stage_ms, runs = plan.stage_ms()
    plan.set_timing(False)

    classes = plan.classes()
    per_class = []
    for ci, (n, su, var) in enumerate(classes):
        unfold_ms = stage_ms[ci, 2] / runs
        bytes_launch = su * 2 * n * 4
        # forward spectra: each station's two float32 traces read, its in-band bins written (16 B each)
        stations = sum(s for s, n_e, _ in specs if n_e == n)
        nb = api.band_bins(api.make_event(1, n, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32))[1]
        spectrum_ms = stage_ms[ci, 0] / runs
        per_class.append({"kernel": api.unfold_kernel_name(api.AU_PREC_FP32, n, var), "variant": var,
                          "n_samples": n,
                          "station_unfolds": int(su),
                          "spectrum_ms": spectrum_ms, "coef_ms": stage_ms[ci, 1] / runs,
                          "spectrum_algorithmic_GBs": stations * (2 * n * 4 + nb * 16) / (spectrum_ms / 1e3) / 1e9,
                          "unfold_ms": unfold_ms,
                          "unfold_algorithmic_GBs": bytes_launch / (unfold_ms / 1e3) / 1e9})
    dom = max(per_class, key=lambda c: c["unfold_ms"])
    achieved = dom["unfold_algorithmic_GBs"]
    traffic = PROFILED_TRAFFIC_BYTES.get((dom["kernel"], dom["station_unfolds"]))
    roofline = {"bound": "hbm", "kernel": dom["kernel"], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "traffic_ratio": None if traffic is None else round(traffic / (dom["station_unfolds"] * 2 * dom["n_samples"] * 4), 4),
                "traffic_source": None if traffic is None else PROFILED_TRAFFIC_SOURCE,
                "bytes_per_unit": "2*N*4 B written per station-unfold",
                "launch_ms": dom["unfold_ms"], "station_unfolds_per_launch": dom["station_unfolds"],
                "measured_copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "per_class": per_class,
                "alu": alu_view(dom), "valu_issue": valu_issue_view(dom)}

    # the timed step: the same plan captured in a hipGraph and replayed back to back
    gplan = api.Plan(tab, specs, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32, flags=args.flags | api.AU_PLAN_GRAPH)
    for _ in range(max(2, args.warmup)):
        gplan.run(volt, efield, counts)
    torch.cuda.synchronize()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    marks[0].record(stream)
    for k in range(args.steps):
        gplan.run(volt, efield, counts)
        marks[k + 1].record(stream)
    torch.cuda.synchronize()
    graph_ms = marks[0].elapsed_time(marks[-1]) / args.steps
    per_step = [marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps)]
    ms_per_step = graph_ms
    value = plan.station_unfolds / (graph_ms / 1e3)
    log("batched fp32 graph replay: %.3f ms/step, %.1f M station-unfolds/s" % (graph_ms, value / 1e6))

    err = parity_sample(grid, table, specs, plan, volt_host, efield)
    cnt = counts.cpu().tolist()
    log("parity sample max per-trace error %.3e; fallback/singular counters %s" % (err, cnt))
    del gplan
    precision = None
    if not args.no_fp32_error:
        tab64f = api.Table(grid, synth.pattern_table(grid, cfg=2).astype(np.complex64).astype(np.complex128))
        precision = fp32_error_report(api, plan, specs, efield, tab64f, volt, dev)
        log("fp32 vs fp64 over %d traces: max %.3e per component, %.3e per station; %s"
            % (precision["traces"], precision["max"], precision["max_station"],
            ", ".join("kappa %g-%g: max %.2e" % (b["kappa"][0], b["kappa"][1], b["max"]) for b in precision["by_kappa"])))
        log("fp32 vs fp64 per component by share of the station peak: %s"
            % ", ".join("%g-%g: max %.2e (%d of %d over 1e-5)" % (b["share"][0], min(b["share"][1], 1.0), b["max"],
                                                                 b["over_1e-5"], b["traces"])
                        for b in precision["by_component_share"]))
        del tab64f
        torch.cuda.empty_cache()

    # ---------------- FP64 plain direction scan ----------------------------
    fp64 = None
    if not args.no_fp64_plain:
        g1 = synth.GRID_COARSE
        t1 = api.Table(g1, synth.pattern_table(g1, cfg=1))
        s1, n1 = 124, 4096
        dirs1 = synth.direction_grid(32, 64)
        v1 = torch.from_numpy(synth.traces(s1, n1, cfg=1, event=0)).to(dev)
        ev = api.make_event(s1, n1, prec=api.AU_PREC_FP64, trace_dtype=api.AU_F64)
        if not args.no_tune and not args.variant_fp64:
            best, ms = api.autotune(t1, ev, n_dir=256, reps=5)
            tuned["fp64_N%d" % n1] = {"variant": best, "shape": api.unfold_variants()[best], "ms": ms}
            log("autotune fp64 N=%d: variant %d" % (n1, best))
        work = torch.empty(api.workspace_bytes(t1, ev, len(dirs1)), dtype=torch.uint8, device=dev)
        del efield
        torch.cuda.empty_cache()
        out1 = torch.empty((len(dirs1), s1, 2, n1), dtype=torch.float64, device=dev)
        settle(lambda: api.unfold_direction_scan(t1, ev, v1, dirs1, out=out1, work=work))
        k1 = max(10, args.steps)
        ev0.record(stream)
        for _ in range(k1):
            api.unfold_direction_scan(t1, ev, v1, dirs1, out=out1, work=work)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms1 = ev0.elapsed_time(ev1) / k1
        su1 = len(dirs1) * s1
        fp64 = {"value": su1 / (ms1 / 1e3), "unit": "station-unfolds/s", "ms_per_call": ms1,
                "workload": "plain FP64 direction scan: 1 event x 124 stations x 4096 float64 samples, "
                            "32x64 directions, complex128 table 1 MHz/5 deg",
                "station_unfolds": su1,
                "output_GBs": su1 * 2 * n1 * 8 / (ms1 / 1e3) / 1e9}
        log("fp64 plain scan: %.3f ms/call, %.1f M station-unfolds/s" % (ms1, fp64["value"] / 1e6))
        fp64["single_event"] = single_event_latency(api, synth, dev)
        log("single event (10 x 2048 FP64, one direction): median %.1f us per call (min %.1f), device %.1f us"
            % (fp64["single_event"]["us_per_call_median"], fp64["single_event"]["us_per_call_min"],
               fp64["single_event"]["device_us_median"]))
        del out1
        torch.cuda.empty_cache()
        # envelope-peak timing over the same scan (two inverse FFTs per station-unfold, 6 values out)
        fp64["envelope_scan"] = envelope_scan_rate(api, t1, ev, v1, dirs1, work, k1, stream)
        v1f = v1.float().contiguous()
        evf = api.make_event(s1, n1, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32)
        workf = torch.empty(api.workspace_bytes(tab, evf, len(dirs1)), dtype=torch.uint8, device=dev)
        fp64["envelope_scan_fp32"] = envelope_scan_rate(api, tab, evf, v1f, dirs1, workf, k1, stream)
        log("envelope scan: fp64 %.1f M, fp32 %.1f M station-unfolds/s"
            % (fp64["envelope_scan"]["value"] / 1e6, fp64["envelope_scan_fp32"]["value"] / 1e6))
        del work, workf, v1f
        fp64["reconstruction"] = reconstruction_latency(api, synth, t1, tab, dev)
        fp64["direction_fit"] = direction_fit_latency(api, synth, t1, dev)
        fp64["direction_fit_fp32"] = direction_fit_latency(api, synth, tab, dev, fp32=True)
        log("direction fit (124 x 4096, 2048 + 100 candidates): fp64 %.3f ms/event, fp32 %.3f ms/event, "
            "max error %.3f / %.3f deg"
            % (fp64["direction_fit"]["ms_per_event"], fp64["direction_fit_fp32"]["ms_per_event"],
               fp64["direction_fit"]["max_angle_err_deg"], fp64["direction_fit_fp32"]["max_angle_err_deg"]))
        rec = fp64["reconstruction"]
        log("reconstruction loop (124 stations x 4096): fp64 %.3f ms/event, fp32 %.3f ms/event; batched %d events: "
            "fp64 %.0f, fp32 %.0f events/s"
            % (rec["fp64"]["ms_per_event"], rec["fp32"]["ms_per_event"], rec["fp64"]["batch"]["events"],
               rec["fp64"]["batch"]["events_per_s"], rec["fp32"]["batch"]["events_per_s"]))
        torch.cuda.empty_cache()

    # ---------------- large batch -----------------------------------------
    large = None
    if not args.no_large_batch:
        large = large_batch_rate(api, synth, tab, grid, table, dev)
        log("large batch: %.3f ms/step (separate stages %.3f), %.1f M station-unfolds/s, %.0f GB/s out (%.1f GB of "
            "distinct inputs generated in %.1f s); FP32 vs oracle on %d units: %.2e per station, %.2e per strong "
            "component"
            % (large["ms_per_step"], large["separate_stages_ms_per_step"], large["value"] / 1e6, large["output_GBs"],
               large["input_GB"],
               large["generation_s"], large["fp32_error_vs_oracle"]["units"],
               large["fp32_error_vs_oracle"]["max_station"], large["fp32_error_vs_oracle"]["max_strong_component"]))

    # ---------------- serving -------------------------------------------
    serving = None
    if not args.no_serving:
        tab64f = api.Table(grid, synth.pattern_table(grid, cfg=2))
        serving = serving_benchmark(api, synth, tab, tab64f, duration_s=args.serve_seconds)
        log("serving: p50 %.3f ms p99 %.3f ms at %.0f events/s (batch %.2f; median ms submit %.3f, "
            "admit->launch %.3f, launch->complete %.3f); plain fp64 loop p50 %.3f p99 %.3f ms"
            % (serving["p50_ms"], serving["p99_ms"], serving["events_per_s"], serving["mean_batch_events"],
               serving["median_ms"]["arrival_to_submit_return"], serving["median_ms"]["admit_to_launch"],
               serving["median_ms"]["launch_to_complete"],
               serving["plain_fp64_loop"]["p50_ms"], serving["plain_fp64_loop"]["p99_ms"]))
        sat = serving["saturated"]
        log("serving saturated: %.0f of %.0f events/s offered, %.1f M station-unfolds/s, mean batch %.2f (max %d), "
            "p50 %.3f ms p99 %.3f ms" % (sat["events_per_s"], sat["offered_events_per_s"],
                                          sat["station_unfolds_per_s"] / 1e6, sat["mean_batch_events"],
                                          sat["max_batch_events"], sat["p50_ms"], sat["p99_ms"]))
        del tab64f

    # ---------------- CPU oracle baseline ---------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(grid, table, specs, plan, volt_host, budget_s=args.cpu_budget)
        log("cpu oracle: %.1f station-unfolds/s on %d threads" % (cpu["value"], cpu["cores"]))

    line = {
        "metric": "station-unfolds/sec FP32-batched vs FP64-plain at 1 GPU; p50/p99 event latency",
        "value": value,
        "unit": "station-unfolds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched FP32 unfolding: %d events, stations U{3..124}, N in {2048,4096}, "
                               "16x16 directions/event, complex64 table 0.5 MHz/1 deg, FP64 det fallback"
                               % len(specs),
                   "events": len(specs), "station_unfolds": int(plan.station_unfolds),
                   "plan_flags": args.flags | api.AU_PLAN_GRAPH, "timed": "hipGraph replay of the plan",
                   "eager_ms_per_step": eager_ms, "step_ms_median": float(np.median(per_step)),
                   "step_ms_min": float(np.min(per_step)), "autotuned": tuned},
        "roofline": roofline,
        "fp64_plain": fp64,
        "large_batch": large,
        "serving": serving,
        "cpu_baseline": cpu,
        "parity_sample_max_err": err,
        "fp32_error_vs_fp64": precision,
        "fallback_singular_bins": cnt,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
