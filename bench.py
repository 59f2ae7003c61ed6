"""Benchmark: Mpix/s per L.A.Cosmic iteration on the mixed-size batch, batched vs per-frame.

A step is one pass of the whole hot path over the batch: niter = 4 iterations
(detection, grow/count, replacement) for all 64 frames of the mixed-size workload
(16 x 800x800, 16 x 1024x1024, 16 x 2048x4096, 16 x 4096x2048; per-frame gain and
read noise), with every iteration forced so that the work is fixed.  Frames are
device-resident before the timed region starts.  The batch plan's launch shapes are
chosen first by the autotuner (crb_plan_autotune, untimed).  The timed region runs the
plan with a pair of HIP events around every launch (on the plan's stream), which gives
the detection kernel's average duration for the roofline.  Then, untimed for the
headline: the same plan with the default shapes, the plan replayed as a captured HIP
graph, incremental detection, the per-frame path (one crb_lacosmic call per frame,
checked identical to the batch), the 4096 x 4096 crowded field through the same paths,
the serving loop on a Poisson request stream, and the FP64 oracle on the host.  rank 0
prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c3|c2|c1]
                  [--no-cpu-baseline] [--no-per-frame] [--no-graph] [--no-incremental]
                  [--no-c3] [--no-tune] [--calib-copy] [--serve-seconds S]
                  [--serve-rate R] [--serve-sweep] [--cpu-plan] [--oracle-parity]
  python bench.py --workload halo|farm|sources      (the framework studies, one JSON line)
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

METRIC = "Mpix/s per L.A.Cosmic iteration (batched vs per-frame); p99 frame latency"
UNIT = "Mpix/s per iteration"
# algorithmic HBM bytes per pixel and iteration of the whole pass: read J (4), write
# J_{k+1} (4), the mask (1)
STEP_BYTES_PER_PIXEL = 9
# the detection's algorithmic lane operations per pixel counted on the mixed batch when
# this figure was frozen; a fraction against it does not move when pruning changes the
# counted work, so it tracks the kernel's speed alone
FROZEN_OPS_PER_PIXEL = 51.34


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _gen(args):
    name, i = args
    from paper_1008_2192_amd import synth
    if name == "c4":
        return synth.c4_frame(i)
    return getattr(synth, name)()


def make_workload(name: str, workers: int):
    if name == "c4":
        jobs = [("c4", i) for i in range(64)]
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(_gen, jobs))
    return [_gen((name, 0))]


def describe(name, frames):
    px = sum(f.img.size for f in frames)
    if name == "c4":
        return {"workload": "mixed-size batch: 64 FP32 frames, 16 each of 800x800, 1024x1024, "
                            "2048x4096, 4096x2048 (HxW), per-frame gain U(1,8), read noise "
                            "U(3,8), 30 stars and 50 cosmic-ray hits per 65536 px; sigclip 4.5, "
                            "sigfrac 0.3, objlim 4, niter 4 (forced)",
                "frames": len(frames), "pixels": px, "niter": 4}
    f = frames[0]
    return {"workload": f"{f.name}: single FP32 frame {f.img.shape[0]}x{f.img.shape[1]}, "
                        f"gain {f.gain}, read noise {f.readnoise}, niter 4 (forced)",
            "frames": 1, "pixels": px, "niter": 4}


KERNEL_SOURCES = ("csrc/detect.hip", "csrc/device_common.h", "csrc/kernels.h", "csrc/medtile.inc")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1008_2192_amd", rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_value(summary, key):
    """A number per detection launch from a committed counter summary (profiles/), if it
    was taken on the current kernel sources (else None)."""
    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def device_items(frames, dev, incremental=False):
    import torch
    items = []
    for f in frames:
        img = torch.from_numpy(f.img).to(dev)
        items.append(dict(img=img, out_clean=torch.empty_like(img),
                          out_mask=torch.empty(img.shape, dtype=torch.uint8, device=dev),
                          gain=f.gain, readnoise=f.readnoise, sky=f.sky, sigclip=f.sigclip,
                          sigfrac=f.sigfrac, objlim=f.objlim, niter=4, early_stop=False,
                          incremental=incremental))
    return items


def time_steps(run, steps, warmup):
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def roofline_record(total_px, det_avg_s, work, step_s, valu_per_launch, traffic):
    """The detection kernel against the lane-op peak (algorithmic ops counted by the
    kernel's own counters), beside two fixed-denominator fractions: ops at a frozen
    per-pixel count, and the whole step's algorithmic HBM bytes against 8 TB/s."""
    from paper_1008_2192_amd import roofline
    work_px = work["work_pixels"] / 4.0
    contrast = work["contrast_tests"] / 4.0
    exact_px = work["exact_med5"] / 4.0
    ops_launch = roofline.detect_ops_per_launch(total_px, exact_px, work_px, contrast)
    achieved = ops_launch / det_avg_s
    o = roofline.detect_ops()
    rec = {"bound": "alu",
           "kernel": "k_detect (detection: a lower bound of med5(J), L+ and the upper bound of S "
                     "it gives everywhere; the med5 network and the FP32 estimate of S with its "
                     "error bound within 4 px of where S may exceed sigclip; med5(S), S' and "
                     "the threshold bits on the work set; the contrast test by counting the med3 "
                     "window where S' > sigclip; binary64 re-evaluation where the bound cannot "
                     "decide)",
           "achieved": round(achieved / 1e12, 3), "peak": round(roofline.ALU_PEAK / 1e12, 3),
           "unit": "Tlane-op/s", "frac": round(achieved / roofline.ALU_PEAK, 4),
           "traffic": traffic,
           "ops_per_launch": round(ops_launch), "ops_per_pixel": round(ops_launch / total_px, 2),
           "dense_ops_per_pixel": round(o["dense"]["total"], 2),
           "ops_per_exact_med5_pixel": round(o["per_exact_pixel"], 2),
           "exact_med5_pixels_per_launch": round(exact_px),
           "ops_per_work_pixel": round(o["per_work_pixel"], 2),
           "ops_per_contrast_test": round(o["per_contrast"], 2),
           "work_pixels_per_launch": round(work_px), "contrast_tests_per_launch": round(contrast),
           "reevaluated_per_launch": round(work["reevaluated"] / 4.0, 2),
           "pixels_per_launch": total_px, "avg_launch_ms": round(det_avg_s * 1e3, 4),
           "frac_frozen_ops": round(FROZEN_OPS_PER_PIXEL * total_px / det_avg_s /
                                    roofline.ALU_PEAK, 4),
           "frozen_ops_per_pixel": FROZEN_OPS_PER_PIXEL,
           "hbm_step_frac": round(STEP_BYTES_PER_PIXEL * total_px * 4 / step_s /
                                  roofline.HBM_PEAK, 4),
           "hbm_step_bytes_per_pixel_iteration": STEP_BYTES_PER_PIXEL}
    rec["issued_lane_op_frac"] = (round(valu_per_launch * 64 / det_avg_s / roofline.ALU_PEAK, 4)
                                  if valu_per_launch else None)
    rec["valu_instructions_per_pixel"] = (round(valu_per_launch * 64 / total_px, 1)
                                          if valu_per_launch else None)
    return rec


def plan_leg(items, total_px, steps, warmup, tune, label, shape=None):
    """Batch plan of `items`: autotuned shapes (unless tune is False; `shape` forces
    one), timed steps with per-launch events, the detection work counters, and the same
    plan at the default shapes.  Returns (record, ms per step, kernel averages, work,
    plan stats, tuning)."""
    from paper_1008_2192_amd import _lib
    plan = _lib.Plan(items, use_graph=False, on_current_stream=True)
    tuned = None
    if shape:
        plan.set_tuning(**shape)
    elif tune:
        tuned = plan.autotune(reps=3, use_cache=True)
        log(f"{label}: autotune {tuned}")
    tuning = plan.get_tuning()
    for _ in range(warmup):
        plan.run()
    plan.set_timing(True)
    step_s = time_steps(plan.run, steps, 0)
    kt = plan.kernel_times()
    stats = plan.stats()
    plan.set_timing(False)
    plan.set_counting(True)
    plan.run()
    work = plan.work_counts()
    plan.set_counting(False)
    rec = {"tuning": tuning}
    # the tuned and the default shapes without per-launch events, for their comparison
    t_s = time_steps(plan.run, steps, warmup)
    rec["tuned_no_events"] = {"ms_per_step": round(t_s * 1e3, 3),
                              "value": round(total_px * 4 / t_s / 1e6, 1)}
    if tuning != _lib.DEFAULT_TUNING:
        plan.set_tuning(**_lib.DEFAULT_TUNING)
        d_s = time_steps(plan.run, steps, warmup)
        plan.set_tuning(**tuning)
    else:
        d_s = t_s
    rec["default"] = {"ms_per_step": round(d_s * 1e3, 3),
                      "value": round(total_px * 4 / d_s / 1e6, 1),
                      "tuned_speedup": round(d_s / t_s, 3)}
    if tuned:
        rec["autotune"] = {"ms": round(tuned["ms"], 4), "default_ms": round(tuned["default_ms"], 4)}
    plan.close()
    kavg = {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items()}
    log(f"{label}: {step_s * 1e3:.3f} ms/step, {total_px * 4 / step_s / 1e6:.0f} Mpix/s per "
        f"iteration; kernel ms " + ", ".join(f"{k} {v[0] / max(v[1], 1):.4f}x{v[1]}"
                                             for k, v in kt.items()))
    return rec, step_s, kt, kavg, work, stats, tuning


def graph_leg(items, tuning, total_px, steps, warmup):
    from paper_1008_2192_amd import _lib
    gplan = _lib.Plan(items, use_graph=True, on_current_stream=True)
    gplan.set_tuning(**tuning)
    g_s = time_steps(gplan.run, steps, warmup)
    gplan.close()
    return {"value": round(total_px * 4 / g_s / 1e6, 1), "ms_per_step": round(g_s * 1e3, 3)}


def per_frame_leg(items, total_px, steps, warmup, tuning=None):
    """One crb_lacosmic call per frame (single-frame launch shapes: the default, or the
    batch plan's tuned detection tile and grow when given).  Its outputs are compared
    with the batch's, which the caller saved."""
    from paper_1008_2192_amd import _lib
    if tuning:
        _lib.set_single_tuning(tuning["tile_h"], tuning["fused"], tuning["grow_h"])
    else:
        _lib.set_single_tuning()

    def step():
        for it in items:
            _lib.lacosmic(it["img"], it["gain"], it["readnoise"], it["sky"], it["sigclip"],
                          it["sigfrac"], it["objlim"], 4, out_clean=it["out_clean"],
                          out_mask=it["out_mask"], early_stop=False)
    try:
        s = time_steps(step, steps, warmup)
    finally:
        _lib.set_single_tuning()
    return s


def c3_leg(args, dev):
    """The 4096 x 4096 crowded field: batch plan (autotuned, events per launch), graph
    replay and the per-frame path; roofline of the detection on this frame."""
    import torch
    from paper_1008_2192_amd import synth
    f = synth.c3()
    items = device_items([f], dev)
    px = f.img.size
    rec, step_s, kt, kavg, work, stats, tuning = plan_leg(items, px, args.steps, args.warmup,
                                                         not args.no_tune, "c3 batch plan",
                                                         parse_shape(args.c3_shape))
    batch_out = (items[0]["out_clean"].clone(), items[0]["out_mask"].clone())
    det_ms, det_n = kt["detect"]
    # a step of this frame is about half a millisecond, so an event around every launch
    # adds a sixth to it: the record's value is the plan timed without them (the event
    # run gives the per-kernel averages and the roofline)
    plain_s = rec["tuned_no_events"]["ms_per_step"] / 1e3
    out = {"workload": "c3: one 4096x4096 FP32 crowded field, 20000 stars (power-law flux), "
                       "1.5% of pixels hit, gain 1.5, read noise 4, niter 4 (forced)",
           "pixels": px, "value": round(px * 4 / plain_s / 1e6, 1),
           "ms_per_step": round(plain_s * 1e3, 3),
           "events_ms_per_step": round(step_s * 1e3, 3), **rec, "kernel_avg_ms": kavg,
           "flagged_pixels": int(stats[0]["n_flagged"])}
    out["roofline"] = roofline_record(px, det_ms / det_n / 1e3, work, step_s,
                                      profiled_value("k_detect_c3_counters.md",
                                                     "valu_instructions_per_launch"),
                                      profiled_value("k_detect_c3_counters.md",
                                                     "traffic_bytes_per_launch"))
    if not args.no_graph:
        out["graph"] = graph_leg(items, tuning, px, args.steps, args.warmup)
    if not args.no_per_frame:
        pf = per_frame_leg(items, px, args.steps, args.warmup)
        same = bool(torch.equal(items[0]["out_clean"], batch_out[0]) and
                    torch.equal(items[0]["out_mask"], batch_out[1]))
        out["per_frame"] = {"ms_per_step": round(pf * 1e3, 3),
                            "value": round(px * 4 / pf / 1e6, 1),
                            "identical_to_batch": same,
                            "batched_speedup": round(pf / plain_s, 3)}
        if "graph" in out:
            out["per_frame"]["graph_speedup"] = round(pf * 1e3 / out["graph"]["ms_per_step"], 3)
        pft = per_frame_leg(items, px, args.steps, args.warmup, tuning)
        out["per_frame_tuned_shapes"] = {"ms_per_step": round(pft * 1e3, 3),
                                         "value": round(px * 4 / pft / 1e6, 1)}
    log(f"c3: {json.dumps({k: v for k, v in out.items() if k != 'roofline'})}")
    del items
    torch.cuda.empty_cache()
    return out


def _pool_frame(args):
    """A frame in electrons (gain 1, read noise 5.5 e-)."""
    from paper_1008_2192_amd import synth
    si, j = args
    H, W = synth.C4_SIZES[si]
    return synth.c1_density_frame(H, W, 5000 + 4 * si + j, 1.0, 5.5).img


def serving_leg(rate, seconds, workers, budget=64 << 30, sweep=False):
    """Requests arrive as a Poisson process; sizes drawn uniformly from the four
    batch sizes, each with its own gain and read noise.  Pixel content comes from a
    pool of 4 frames per size generated in electrons (the request's seed picks one)
    and divided by the request's gain, which keeps generation time bounded while the
    noise level matches the request's parameters.  Served on the same trace by
    continuous batching (64 slots) and one frame at a time (1 slot), from host buffers
    (pageable), and from device-resident inputs (the host link out of the way)."""
    import torch
    from paper_1008_2192_amd import serving, synth
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        pool = list(ex.map(_pool_frame, [(si, j) for si in range(4) for j in range(4)]))
    sizes = list(synth.C4_SIZES)

    def trace(r, s):
        reqs = synth.c5_stream(rate=r, duration=s)
        frames, params = [], []
        for q in reqs:
            si = sizes.index((q.H, q.W))
            frames.append((pool[4 * si + (q.seed % 4)] / np.float32(q.gain)).astype(np.float32))
            params.append(dict(gain=q.gain, readnoise=q.readnoise, niter=4))
        return [q.t_arrival for q in reqs], frames, params

    arrivals, frames, params = trace(rate, seconds)
    out = {"trace": f"Poisson arrivals at {rate:g} frames/s over {seconds:g} s "
                    f"({len(arrivals)} requests), sizes uniform over 800x800, 1024x1024, "
                    f"2048x4096, 4096x2048, per-request gain U(1,8) and read noise U(3,8), "
                    f"niter 4 with early stop, HBM budget {budget >> 30} GiB; latency from "
                    f"submit to result in host memory (host inputs) or to the result on the "
                    f"device (device inputs)"}
    dframes = [torch.from_numpy(f).cuda() for f in frames]
    for name, slots, src in (("continuous", 64, frames), ("sequential", 1, frames),
                             ("continuous_device", 64, dframes),
                             ("sequential_device", 1, dframes)):
        srv = serving.Server(budget, max_slots=slots)
        srv.submit(pool[0], 1.0, 5.0)               # warm-up request
        srv.drain()
        res = serving.replay(srv, arrivals, src, params)
        srv.close()
        out[name] = res.summary()
        log(f"serving {name}: {out[name]}")
    # saturation: the whole trace (up to 256 requests) arrives at once
    n = min(len(frames), 256)
    for name, slots, src in (("burst_continuous_device", 64, dframes),
                             ("burst_sequential_device", 1, dframes),
                             ("burst_continuous", 64, frames), ("burst_sequential", 1, frames)):
        srv = serving.Server(budget, max_slots=slots)
        res = serving.replay(srv, [0.0] * n, src[:n], params[:n])
        srv.close()
        out[name] = res.summary()
        log(f"serving {name}: {out[name]}")
    if sweep:
        # load sweep with device-resident inputs, continuous vs sequential, and a
        # reduced HBM budget that makes admission bind
        out["sweep"] = []
        for r in (40.0, 160.0, 640.0, 2560.0):
            a2, f2, p2 = trace(r, min(seconds, 600.0 / r))
            d2 = [torch.from_numpy(f).cuda() for f in f2]
            row = {"rate": r, "requests": len(a2)}
            for name, slots, bud in (("continuous", 64, budget), ("sequential", 1, budget),
                                     ("continuous_2GiB", 64, 2 << 30)):
                srv = serving.Server(bud, max_slots=slots)
                res = serving.replay(srv, a2, d2, p2)
                srv.close()
                row[name] = res.summary()
            log(f"serving sweep: {row}")
            out["sweep"].append(row)
            del d2
    del dframes
    torch.cuda.empty_cache()
    return out


def cpu_baseline(frames_for_cpu):
    """The FP64 oracle as it stands, single-threaded, on a bounded sample; returns the
    baseline record, the results (for the all-cores run's exactness check) and the
    wall time."""
    from oracle import ref
    t0 = time.perf_counter()
    px_iter = 0
    results = []
    for f in frames_for_cpu:
        r = ref.lacosmic(f.img, f.gain, f.readnoise, f.sky, f.sigclip, f.sigfrac, f.objlim, 4,
                         early_stop=False)
        results.append((r["clean"], r["mask"]))
        px_iter += f.img.size * 4
    dt = time.perf_counter() - t0
    rec = {"value": round(px_iter / dt / 1e6, 4), "unit": UNIT, "cores": 1, "kind": "oracle",
           "sample": f"{len(frames_for_cpu)} frame(s) of "
                     f"{'+'.join(f'{f.img.shape[0]}x{f.img.shape[1]}' for f in frames_for_cpu)}"
                     f" px, 4 forced iterations, {dt:.1f} s on one host thread (nproc "
                     f"{os.cpu_count()})"}
    return rec, results, dt


def cpu_all_cores(frames_for_cpu, single_results, single_s):
    """The CRBLASTER arrangement on the host (Section 6.2): each sample frame split in
    2-D into about two rectangles per worker, extended by a border of 8 px per iteration
    (so the stitched interiors equal the whole-frame result), the extended subimages
    cleaned by independent workers on the host cores."""
    from oracle import partition
    workers = partition.host_workers()
    t0 = time.perf_counter()
    exact, splits = True, []
    for f, (c1, m1) in zip(frames_for_cpu, single_results):
        r = partition.lacosmic_partitioned(f.img, f.gain, f.readnoise, f.sky, f.sigclip,
                                           f.sigfrac, f.objlim, 4, workers=workers)
        exact &= bool(np.array_equal(r["clean"], c1) and np.array_equal(r["mask"], m1))
        splits.append(f"{r['split'][0]}x{r['split'][1]}")
    dt = time.perf_counter() - t0
    px_iter = sum(f.img.size for f in frames_for_cpu) * 4
    speedup = single_s / dt
    return {"value": round(px_iter / dt / 1e6, 4), "unit": UNIT, "cores": workers,
            "kind": "oracle", "speedup": round(speedup, 2),
            "efficiency": round(speedup / workers, 3), "identical_to_single": exact,
            "sample": f"the same frames split {'/'.join(splits)} with a 32-pixel border, "
                      f"{workers} worker threads each cleaning its own subimages, "
                      f"{dt:.2f} s wall"}


def cpu_plan():
    """The oracle timing plan: single-threaded on the 256^2, 800^2 (median of 3) and
    4096^2 (once) frames, all iterations forced, and the 4096^2 frame as bordered
    subimages on all host cores."""
    from oracle import partition, ref
    from paper_1008_2192_amd import synth
    out = {"host_threads": partition.host_workers(), "nproc": os.cpu_count()}
    try:
        out["lscpu_model"] = next(l.split(":", 1)[1].strip()
                                  for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        out["lscpu_model"] = None
    for name, reps in (("c1", 3), ("c2", 3), ("c3", 1)):
        f = getattr(synth, name)()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            ref.lacosmic(f.img, f.gain, f.readnoise, f.sky, f.sigclip, f.sigfrac, f.objlim, 4,
                         early_stop=False)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        out[name] = {"pixels": f.img.size, "single_thread_s": round(t, 3),
                     "value": round(f.img.size * 4 / t / 1e6, 4), "runs": reps}
        log(f"cpu plan {name}: {out[name]}")
        if name == "c3":
            r = partition.lacosmic_partitioned(f.img, f.gain, f.readnoise, f.sky, f.sigclip,
                                               f.sigfrac, f.objlim, 4)
            sp = t / r["wall_s"]
            out["c3_all_cores"] = {"wall_s": round(r["wall_s"], 3), "workers": r["workers"],
                                   "split": f"{r['split'][0]}x{r['split'][1]}",
                                   "value": round(f.img.size * 4 / r["wall_s"] / 1e6, 4),
                                   "speedup": round(sp, 2),
                                   "efficiency": round(sp / r["workers"], 3)}
            log(f"cpu plan c3 all cores: {out['c3_all_cores']}")
    return out


def oracle_parity(frames, items):
    """Every frame of the batch against the oracle run as bordered subimages on all
    host cores: mask mismatches and cleaned pixels beyond 1e-5 relative, per frame."""
    from oracle import partition
    t0 = time.perf_counter()
    n_mask = n_clean = 0
    worst = 0.0
    for i, (f, it) in enumerate(zip(frames, items)):
        if i % 8 == 0:
            log(f"oracle parity: frame {i} of {len(frames)}, {time.perf_counter() - t0:.1f} s")
        r = partition.lacosmic_partitioned(f.img, f.gain, f.readnoise, f.sky, f.sigclip,
                                           f.sigfrac, f.objlim, 4)
        gm = it["out_mask"].cpu().numpy()
        gc = it["out_clean"].cpu().numpy().astype(np.float64)
        zero = r["clean"] == 0.0
        rel = np.abs(gc - r["clean"]) / np.where(zero, 1.0, np.abs(r["clean"]))
        n_mask += int((gm != r["mask"]).sum())
        n_clean += int((rel > 1e-5).sum()) + int((gc[zero] != 0.0).sum())
        worst = max(worst, float(rel.max()))
    dt = time.perf_counter() - t0
    return {"frames": len(frames), "pixels": int(sum(f.img.size for f in frames)),
            "mask_mismatches": n_mask, "clean_beyond_1e-5": n_clean,
            "max_rel_clean_diff": worst, "oracle_wall_s": round(dt, 1),
            "oracle_threads": partition.host_workers()}


# ---- framework studies: the paper's partition border, framework probes, list outputs

def halo_mode(niter=4):
    """Border (halo) sweep of the paper's partitioned run (Section 6.2: 6 px is the
    smallest border without artifacts): mask and cleaned pixels differing from the
    unpartitioned run, per partition and border."""
    import torch
    from paper_1008_2192_amd import _lib, synth
    out = {"workload": "halo", "niter": niter, "rows": []}
    for f in (synth.c2(), synth.c3()):
        img = torch.from_numpy(f.img).to("cuda")
        c0, m0 = _lib.lacosmic(img, f.gain, f.readnoise, niter=niter)
        torch.cuda.synchronize()
        for ny, nx in ((2, 4), (6, 6), (1, 36), (7, 7)):
            for b in (0, 2, 4, 6, 8, 16, 32):
                c, m = _lib.lacosmic_partitioned(img, f.gain, f.readnoise, ny, nx, b,
                                                 niter=niter)
                torch.cuda.synchronize()
                out["rows"].append(dict(frame=f.name, partition=f"{ny}x{nx}", border=b,
                                        mask_diff=int((m != m0).sum().item()),
                                        clean_diff=int((c != c0).sum().item()),
                                        flagged=int(m0.sum().item())))
        del img
    return out


def farm_mode(band_rows=1):
    """The paper's POISSON and WAITER probes (Sections 6.3.2-6.3.3) on 750x750 images
    of 24.3 and 137: speedup and efficiency against the number of actors (waves)."""
    import torch
    from paper_1008_2192_amd import _lib
    out = {"workload": "farm", "band_rows": band_rows, "rows": []}
    for name, kind, value in (("POISSON", _lib.CRB_WORK_POISSON, 24.3),
                              ("WAITER", _lib.CRB_WORK_WAITER, 137.0)):
        x = torch.full((750, 750), value, device="cuda")
        _lib.work_run(kind, x, workers=64, band_rows=band_rows)
        torch.cuda.synchronize()
        t1 = None
        for n in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096):
            best = None
            for _ in range(3):
                s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s.record()
                _lib.work_run(kind, x, seed=1, workers=n, band_rows=band_rows)
                e.record()
                torch.cuda.synchronize()
                best = s.elapsed_time(e) if best is None else min(best, s.elapsed_time(e))
            t1 = best if t1 is None else t1
            out["rows"].append(dict(work=name, workers=n, ms=round(best, 4),
                                    speedup=round(t1 / best, 2),
                                    efficiency=round(t1 / best / n, 4)))
    return out


def sources_mode(tiles=None, workers=None, frames=None):
    """The SOURCES work function (Section 7: actors returning structures) on the
    4096x4096 crowded field and on that field tiled 4 x 4 (1 GiB): algorithmic bytes
    (4 B per pixel + 40 B per source) per launch against 8 TB/s, over tile shapes and
    actor counts (or the ones given)."""
    import torch
    from paper_1008_2192_amd import _lib, synth
    f = synth.c3()
    sky = 200.0 / 1.5
    t = sky + 5.0 * np.sqrt(200.0 + 16.0) / 1.5
    out = {"workload": "sources", "rows": []}
    for name in frames or ("4096x4096", "16384x16384"):
        frame = f.img if name == "4096x4096" else np.tile(f.img, (4, 4))
        x = torch.from_numpy(frame).cuda()
        res = _lib.farm_sources(x, t, sky, 2, 3, capacity=1 << 22)
        torch.cuda.synchronize()
        n_src = int(res.count.item())
        alg = 4.0 * frame.size + 40.0 * n_src
        for th, tw in tiles or ((16, 64), (32, 64), (64, 64), (32, 128), (8, 256)):
            for w in workers or (1024, 2048, 4096, 8192, 16384):
                evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                       for _ in range(10)]
                _lib.farm_sources(x, t, sky, 2, 3, workers=w, tile_h=th, tile_w=tw, out=res)
                for a, b in evs:
                    a.record()
                    _lib.farm_sources(x, t, sky, 2, 3, workers=w, tile_h=th, tile_w=tw, out=res)
                    b.record()
                torch.cuda.synchronize()
                ms = sorted(a.elapsed_time(b) for a, b in evs)[5]
                gbs = alg / (ms * 1e-3) / 1e9
                out["rows"].append(dict(frame=name, tile=f"{th}x{tw}", workers=w,
                                        ms=round(ms, 4), sources=n_src, gbs=round(gbs, 1),
                                        frac=round(gbs / 8000.0, 3)))
        del x, res
        torch.cuda.empty_cache()
    return out


def parse_shape(text):
    if not text:
        return None
    th, pe, fu, gh = (int(v) for v in text.split(","))
    return dict(tile_h=th, persistent=pe, fused=fu, grow_h=gh)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4",
                    choices=["c1", "c2", "c3", "c4", "halo", "farm", "sources"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-frame", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-incremental", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 4096x4096 record")
    ap.add_argument("--no-tune", action="store_true", help="default launch shapes, no autotune")
    ap.add_argument("--shape", default=None,
                    help="launch shapes tile_h,persistent,fused,grow_h instead of the "
                         "autotuner's (e.g. 32,1,0,32)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run 1 GiB device copies, wide (torch) and by 4-byte buffer "
                         "loads (counter calibration)")
    ap.add_argument("--c3-shape", default=None,
                    help="launch shapes of the 4096x4096 record instead of the autotuner's")
    ap.add_argument("--sources-tile", default=None, help="sources study: one tile, e.g. 64x64")
    ap.add_argument("--sources-workers", type=int, default=None,
                    help="sources study: one actor count")
    ap.add_argument("--sources-frame", default=None, choices=["4096x4096", "16384x16384"])
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the Poisson request trace (0 skips serving)")
    ap.add_argument("--serve-rate", type=float, default=40.0)
    ap.add_argument("--serve-sweep", action="store_true",
                    help="serving load sweep (40 to 2560 frames/s) and a 2 GiB budget")
    ap.add_argument("--cpu-plan", action="store_true",
                    help="the oracle timing plan: 256^2, 800^2, 4096^2 single-threaded and "
                         "4096^2 on all host cores")
    ap.add_argument("--oracle-parity", action="store_true",
                    help="every pixel of every batch frame against the oracle on all host "
                         "cores")
    args = ap.parse_args()
    # launch shapes chosen by the autotuner on MI355X for the batch layouts timed here
    # (a tune cache keyed by device and layout; other layouts or devices are tuned live)
    os.environ.setdefault("CRB_TUNE_CACHE", os.path.join(ROOT, "paper_1008_2192_amd",
                                                         "tune_cache.txt"))

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (frames shard across GPUs by "
              "whole frames; no multi-GPU path is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1008_2192_amd import _lib

    _lib.lib()                     # fail loudly if the HIP library is missing
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.workload in ("halo", "farm", "sources"):
        if args.workload == "sources":
            out = sources_mode(
                [tuple(int(v) for v in args.sources_tile.split("x"))] if args.sources_tile
                else None,
                [args.sources_workers] if args.sources_workers else None,
                [args.sources_frame] if args.sources_frame else None)
        else:
            out = {"halo": halo_mode, "farm": farm_mode}[args.workload]()
        print(json.dumps(out), flush=True)
        return
    t0 = time.perf_counter()
    frames = make_workload(args.workload, args.workers)
    log(f"generated {len(frames)} frame(s) in {time.perf_counter() - t0:.1f} s")
    # every leg runs on one stream of the benchmark's own (plans, graphs and the
    # per-frame calls alike), so no leg pays for cross-stream waits
    with torch.cuda.stream(torch.cuda.Stream(device=dev)):
        run(args, dev, frames)


def run(args, dev, frames):
    import torch
    from paper_1008_2192_amd import _lib

    items = device_items(frames, dev)
    torch.cuda.synchronize()
    total_px = sum(f.img.size for f in frames)
    px_iter = total_px * 4

    # ---- timed region: the autotuned batch plan, events around every launch -----
    rec, step_s, kt, kavg, work, stats, tuning = plan_leg(items, total_px, args.steps,
                                                         args.warmup, not args.no_tune,
                                                         "batch plan", parse_shape(args.shape))
    value = px_iter / step_s / 1e6
    det_ms, det_n = kt["detect"]
    summary = "k_detect_batch64_counters.md" if args.workload == "c4" else None
    roof = roofline_record(total_px, det_ms / det_n / 1e3, work, step_s,
                           profiled_value(summary, "valu_instructions_per_launch")
                           if summary else None,
                           profiled_value(summary, "traffic_bytes_per_launch")
                           if summary else None)
    roof["kernel_avg_ms"] = kavg
    roof["kernel_note"] = ("detection evaluates every pixel at every iteration; the grow "
                           "visits the strips within reach of A, and from iteration 2 on the "
                           "replacement recomputes only flagged pixels near a new flag "
                           "(elsewhere their results equal what the frame holds)")
    out = {"metric": METRIC, "value": round(value, 1), "unit": UNIT, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_s * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64", "data": "synthetic",
           "config": describe(args.workload, frames), "roofline": roof}
    out["flagged_pixels"] = int(sum(s["n_flagged"] for s in stats))
    out.update(rec)
    batch_out = [(it["out_clean"].clone(), it["out_mask"].clone()) for it in items]

    if args.oracle_parity:
        out["oracle_parity"] = oracle_parity(frames, items)
        log(f"oracle parity: {out['oracle_parity']}")

    if not args.no_graph:
        out["graph"] = graph_leg(items, tuning, total_px, args.steps, args.warmup)
        log(f"graph replay: {out['graph']}")

    if not args.no_incremental:
        inc_items = [dict(it, incremental=True) for it in items]
        iplan = _lib.Plan(inc_items, use_graph=False, on_current_stream=True)
        iplan.set_tuning(**tuning)
        for _ in range(args.warmup):
            iplan.run()
        iplan.set_timing(True)
        idt = time_steps(iplan.run, args.steps, 0)
        ikt = iplan.kernel_times()
        iplan.set_timing(False)
        iplan.close()
        out["incremental"] = {
            "value": round(px_iter / idt / 1e6, 1), "ms_per_step": round(idt * 1e3, 3),
            "detect_ms_per_step": round(ikt["detect"][0] / args.steps, 3),
            "note": "from iteration 2 on, detection re-runs only on tiles whose codes can "
                    "change (J changed within 4 px); results identical to the headline's"}
        log(f"incremental: {out['incremental']}")

    if not args.no_per_frame:
        pdt = per_frame_leg(items, total_px, args.steps, args.warmup)
        same = all(torch.equal(it["out_clean"], c) and torch.equal(it["out_mask"], m)
                   for it, (c, m) in zip(items, batch_out))
        pf = px_iter / pdt / 1e6
        out["per_frame"] = {"value": round(pf, 1), "ms_per_step": round(pdt * 1e3, 3),
                            "batched_speedup": round(value / pf, 3),
                            "identical_to_batch": same}
        if "graph" in out:
            out["per_frame"]["graph_speedup"] = round(out["graph"]["value"] / pf, 3)
        log(f"per-frame: {out['per_frame']}")
    del batch_out

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        for _ in range(3):
            _lib.debug_copy_b32(src, dst)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 2 * src.numel() * 4
        del src, dst

    if args.workload == "c4" and not args.no_c3:
        del items
        torch.cuda.empty_cache()
        items = None
        out["c3"] = c3_leg(args, dev)

    if args.serve_seconds > 0 and args.workload == "c4":
        items = None
        torch.cuda.empty_cache()
        out["serving"] = serving_leg(args.serve_rate, args.serve_seconds, args.workers,
                                     sweep=args.serve_sweep)

    if not args.no_cpu_baseline:
        sample = [f for f in frames if f.img.shape == (800, 800)][:2] or frames[:1]
        if args.workload == "c3":
            from paper_1008_2192_amd import synth
            sample = [synth.c3(size=512)]
        out["cpu_baseline"], single, single_s = cpu_baseline(sample)
        log(f"cpu baseline: {out['cpu_baseline']}")
        out["cpu_all_cores"] = cpu_all_cores(sample, single, single_s)
        log(f"cpu all cores: {out['cpu_all_cores']}")
    if args.cpu_plan:
        out["cpu_plan"] = cpu_plan()

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
