#!/usr/bin/env python3
"""Throughput and latency of the tracking hot path on one MI355X.

Workload (the 256x256 streaming case): 10,000 frames of 256x256 12-bit
pixels (uint16) holding an Airy ring pattern (first zero at 8 px, peak 4000
photons, background 50) with Poisson noise, displaced by a random walk with
N(0, 0.3 px) steps; upsampling factor u = 100 on the 1.5-px window.

A "step" is one batched call of the whole path (correlation FFTs, integer
peak, upsampled matrix DFT, FP64 Newton) over all frames, inputs already
resident in HBM; by default its launch chunks alternate between two streams
(--streams 2; the one-stream figure is reported beside it).  Also reported: the plain per-frame path (one call and one
synchronisation per frame), the same with a captured hipGraph, the
roofline of the dominant kernel from HIP events, and the FP64 CPU oracle
timed on a bounded sample of the same frames (also used to check the GPU
results to the 1e-3 px bar).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/sec + p50/p99 per-frame latency at 256×256, batched vs plain, at ≤1e-3 px"

# MI355X datasheet peaks (dense)
PEAK_TFLOPS = {"fp32": 157.3, "bf16x2": 2500.0, "fp16x2": 2500.0}
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel_tag):
    """Per-frame HBM bytes of a kernel from the committed rocprofv3 counter
    summary, if the kernel source is unchanged since the counters were taken
    (the summary records the source's sha256); else None."""
    import glob
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_2310_08770_amd", "csrc", "updft.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            m = re.search(r"traffic kernel=(\S+) bytes_per_frame=(\d+) source_sha256=([0-9a-f]+)", line)
            if m and m.group(1) == kernel_tag and m.group(3) == sha:
                return int(m.group(2))
    return None


def updft_flops_per_frame(n, M, precision):
    """Algorithmic flops of the upsampled matrix DFT per frame: the complex
    Stage A product (M x N by N x H) and the real-part Stage B product
    (M x 2H by 2H x M); split precision runs three products per term."""
    H = n // 2 + 1
    f = 8.0 * M * n * H + 4.0 * M * M * H
    return f * (3 if precision in ("bf16x2", "fp16x2") else 1)


# ---------------------------------------------------------------- CPU baseline
def _oracle_worker(args):
    from threadpoolctl import threadpool_limits

    frames, ref, u = args
    from oracle import ccpt_oracle as O

    out = []
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for f in frames:
            t1 = time.perf_counter()
            r = O.track(f, ref, u)
            out.append((r["d"], r["p"], r["status"], r["d_grid"], r["grid_gap"], r["grid_ac"],
                        time.perf_counter() - t1))
        dt = time.perf_counter() - t0
    return out, dt


def cpu_model():
    """The host CPU's model name from /proc/cpuinfo (else the platform's)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def gpu_clocks():
    """The GPU's current clocks as rocm-smi reports them (a read-only query in a
    child process), or None where the tool is missing or prints no JSON."""
    import shutil
    import subprocess
    # not under rocprofv3: its preloaded tool would initialise the GPU in the
    # child before the tool's own program starts
    if any(k.startswith("ROCPROF") for k in os.environ) or "rocprof" in os.environ.get("LD_PRELOAD", ""):
        return None
    exe = shutil.which("rocm-smi") or "/opt/rocm/bin/rocm-smi"
    try:
        r = subprocess.run([exe, "--showclocks", "--json"], capture_output=True, text=True, timeout=30)
        data = json.loads(r.stdout)
    except Exception:  # noqa: BLE001
        return None
    cards = [v for k, v in sorted(data.items()) if k.startswith("card") and isinstance(v, dict)]
    if not cards:
        return None
    import re
    keep = {}
    for k, v in cards[0].items():  # e.g. "sclk clock speed:": "(2388Mhz)"
        m = re.search(r"(\d+)\s*mhz", str(v), re.I)
        name = k.split()[0].lower() if k else ""
        if m and "speed" in k.lower() and name in ("sclk", "mclk", "fclk", "socclk"):
            keep[f"{name}_mhz"] = int(m.group(1))
    return keep or None


def cpu_baseline(frames, ref, u, sample, cores):
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp

    ref64 = np.asarray(ref, np.float32).astype(np.float64)
    sub = frames[:sample]
    parts = np.array_split(np.arange(len(sub)), cores)
    jobs = [([sub[i] for i in p], ref64, u) for p in parts if len(p)]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(len(jobs), mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(_oracle_worker, jobs))
    wall = time.perf_counter() - t0
    col = lambda j: np.concatenate([np.array([r[j] for r in part]) for part, _ in res])  # noqa: E731
    cpu_s = sum(dt for _, dt in res)
    return dict(d=col(0), p=col(1), status=col(2), d_grid=col(3), grid_gap=col(4), grid_ac=col(5),
                frame_s=col(6), wall=wall, cpu_s=cpu_s, cores=len(jobs))


def cpu_one_core(frames, ref, u, sample):
    """The oracle in this process on one core: per-frame times of `sample` frames."""
    ref64 = np.asarray(ref, np.float32).astype(np.float64)
    out, dt = _oracle_worker((frames[:sample], ref64, u))
    return np.array([r[6] for r in out]), dt


# ---------------------------------------------------------------- GPU legs
def time_batched(tr, frames_t, rois, out, steps, warmup, torch):
    for _ in range(warmup):
        tr.track(None, out=out, rois=rois)
    torch.cuda.synchronize()
    tr.stage_times(reset=True) if tr.options.flags & 2 else None
    lat = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        tr.track(None, out=out, rois=rois)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    return total, np.array(lat)


def time_plain(tr, frames_t, count, torch):
    out = torch.empty((1, 72), dtype=torch.uint8, device=frames_t.device)
    lat = []
    for i in range(min(count, frames_t.shape[0])):
        rois = tr.rois(frames_t[i:i + 1])
        t0 = time.perf_counter()
        tr.track(None, out=out, rois=rois)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    return np.array(lat)


def _sync_time(fn, reps, torch):
    """Wall time per call of fn() over reps calls, synchronised on both sides."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def leg_uneven_rois(dev, torch, Tracker):
    """4096 ROIs of seven sizes (32..256) with their own references, one
    batched FP32 call: size groups one after another with the default plans,
    the default (concurrent size groups, default plans), and the plans and
    lane count chosen by the autotuner timing this mixed call."""
    from synth import frames as S
    w = S.config3(4096)
    refs = [torch.from_numpy(r.astype(np.float32)).to(dev) for r in w.refs]
    fr = [torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in w.frames]
    ids = [int(i) for i in w.ref_ids]
    out = {}
    ref_res = None
    for name in ("serial_groups", "default", "autotuned"):
        tr = Tracker(upsample=w.u)
        tr.set_reference(refs)
        rois = tr.rois(fr, ids)
        res = torch.empty((len(fr), 72), dtype=torch.uint8, device=dev)
        if name == "serial_groups":
            tr.lanes(1)
        if name == "autotuned":
            tr.autotune_batch(rois=rois)
        dt = _sync_time(lambda: tr.track(None, out=res, rois=rois), 10, torch)
        out[name] = dict(rois_per_s=round(len(fr) / dt, 1), ms_per_call=round(dt * 1e3, 3),
                         lanes=tr.lanes())
        if name == "autotuned":
            out[name]["plans"] = {int(n): tr.plan(int(n)) for n in sorted(set(int(x) for x in w.meta["sizes"]))}
        if ref_res is None:
            ref_res = res.clone()
        else:
            out[name]["bit_identical_to_serial"] = bool(torch.equal(res, ref_res))
        tr.close()
    return out


def leg_gauss512(dev, torch, Tracker):
    """2048 frames of 512x512 at u = 200 (M = 300): batched split precision
    against batched FP32."""
    from synth import frames as S
    w = S.config4(2048)
    fr = torch.from_numpy(np.stack(w.frames)).to(dev)
    ref = torch.from_numpy(w.refs[0].astype(np.float32)).to(dev)
    out = {}
    for prec in ("bf16x2", "fp32"):
        tr = Tracker(upsample=w.u, precision=prec)
        tr.set_reference(ref)
        tr.autotune(512, fr.shape[0])
        rois = tr.rois(fr)
        res = torch.empty((fr.shape[0], 72), dtype=torch.uint8, device=dev)
        dt = _sync_time(lambda: tr.track(None, out=res, rois=rois), 5, torch)
        out[prec] = dict(frames_per_s=round(fr.shape[0] / dt, 1), ms_per_call=round(dt * 1e3, 3))
        tr.close()
    return out


def leg_grad128(dev, torch, Tracker):
    """1024 frames of 128x128 (float32 photon counts): forward + backward
    (frame and template gradients) throughput, and the time of one Adam step
    of the template optimisation."""
    from synth import frames as S
    from paper_2310_08770_amd.autograd import optimise_template
    w = S.config5(1024)
    fr = torch.from_numpy(np.stack(w.frames)).to(dev)
    ref = torch.from_numpy(w.refs[0].astype(np.float32)).to(dev)
    tr = Tracker(upsample=w.u)
    tr.set_reference(ref)
    g_d = torch.randn((fr.shape[0], 2), dtype=torch.float64, device=dev)

    def fwd_bwd():
        o = tr.track(fr)
        tr.track_grad(fr, o, g_d, None)

    dt = _sync_time(fwd_bwd, 10, torch)
    shifts = torch.from_numpy(w.shifts - w.shifts[0]).to(dev)
    ref0 = torch.from_numpy(np.maximum(w.frames[0], 1.0).astype(np.float32)).to(dev)
    optimise_template(fr, shifts, ref0, tr, steps=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, losses = optimise_template(fr, shifts, ref0, tr, steps=20)
    torch.cuda.synchronize()
    adam = (time.perf_counter() - t0) / 20
    tr.close()
    return dict(fwd_bwd_frames_per_s=round(fr.shape[0] / dt, 1), fwd_bwd_ms=round(dt * 1e3, 3),
                adam_step_ms=round(adam * 1e3, 3), loss_first=losses[0], loss_last=losses[-1])


# Table I of the paper: CC-SN throughput on an RTX 3080 (images/s) for its
# image sizes (width x height) and u = 128, 256, 512, 1024; context for the
# same settings here.  Keys are (rows, columns).
TABLE1_RTX3080 = {
    (128, 256): {128: 1636, 256: 811, 512: 325, 1024: 91.9},
    (256, 256): {128: 981, 256: 432, 512: 189, 1024: 67.0},
    (256, 512): {128: 670, 256: 322, 512: 168, 1024: 58.6},
    (512, 512): {128: 348, 256: 169, 512: 93, 1024: 31.1},
    (128, 1024): {128: 717, 256: 360, 512: 227, 1024: 85.3},
}


def leg_table1(dev, torch, Tracker):
    """CC-SN (eps = 200) batched split-precision throughput at Table I's five
    image sizes (rows x columns 128x256, 256x256, 256x512, 512x512,
    128x1024: the paper's width x height) for u = 128 .. 1024 (grids of 192
    to 1536 points a side), 512 Airy-ring frames each; the rectangles also
    held tall (transposed input) at u = 128."""
    from synth import frames as S
    out = {}
    cases = [(shape, u) for shape in TABLE1_RTX3080 for u in (128, 256, 512, 1024)]
    cases += [((nx, ny), 128) for (ny, nx) in TABLE1_RTX3080 if ny != nx]
    made = {}
    for (ny, nx), u in cases:
        if (ny, nx) not in made:
            made.clear()
            w = S.table1_frames(ny, nx, 512)
            made[(ny, nx)] = (torch.from_numpy(np.stack(w.frames)).to(dev),
                              torch.from_numpy(w.refs[0].astype(np.float32)).to(dev))
        fr, ref = made[(ny, nx)]
        res = torch.empty((fr.shape[0], 72), dtype=torch.uint8, device=dev)
        tr = Tracker(upsample=u, precision="bf16x2", mode="ccsn", eps=200.0)
        tr.set_reference(ref)
        rois = tr.rois(fr)
        dt = _sync_time(lambda: tr.track(None, out=res, rois=rois), 3, torch)
        rec = dict(frames_per_s=round(fr.shape[0] / dt, 1))
        paper = TABLE1_RTX3080.get((ny, nx), {}).get(u)
        if paper is not None:
            rec["paper_rtx3080_images_per_s"] = paper
        out[f"{ny}x{nx}_u{u}"] = rec
        tr.close()
    return out


def leg_fig1(dev, torch, Tracker):
    """The accuracy study of Fig. 1 at its centre point: 512x512 frames,
    u = 512, w0 = 32, the three image types, 256 frames each; the spread of
    CC-U and CC-SN over the Cramer-Rao bound and the tracking rate."""
    from paper_2310_08770_amd.accuracy import run_condition
    from synth import frames as S
    out = {}
    for kind in S.FIG1_KINDS:
        r = run_condition(kind, 32, 1.0, 256, device=dev.index or 0)
        out[kind] = {m: dict(over_crb=round(r[m]["over_crb"], 3), over_snl=round(r[m]["over_snl"], 3),
                             frames_per_s=r[m]["frames_per_s"]) for m in ("ccu", "ccsn")}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=10000)
    ap.add_argument("--precision", default="bf16x2", choices=["fp32", "bf16x2", "fp16x2"])
    ap.add_argument("--plain-frames", type=int, default=2000)
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-frame legs")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the two-stream leg and the other workloads (mixed ROIs, 512x512 u=200, "
                         "128x128 gradients, Table I, Fig. 1)")
    ap.add_argument("--no-tune", action="store_true", help="skip the chunk autotuner")
    ap.add_argument("--chunk", type=int, default=768,
                    help="frames per launch chunk of the headline leg (768, three frames per CU, as in "
                         "the committed rocprofv3 summary); 0: the autotuner's choice")
    ap.add_argument("--streams", type=int, default=2, choices=[1, 2],
                    help="streams of the timed headline leg: 2 runs alternate launch chunks on two streams "
                         "(CCPT_FLAG_STREAMS: one chunk's DFT overlaps the next chunk's correlation; results "
                         "bit-identical to one stream); the per-kernel roofline always comes from a one-stream "
                         "pass with HIP events around each launch")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain copy of this many MiB first (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the path runs one GPU's share "
              "of the frames, and sharding frames across GPUs is not built", file=sys.stderr)
        sys.exit(2)

    from synth import frames as S

    t0 = time.perf_counter()
    w = S.config2(args.frames)
    frames = np.stack(w.frames)
    ref = w.refs[0].astype(np.float32)
    n, N = frames.shape[0], frames.shape[1]
    log(f"[bench] generated {n} frames {N}x{N} in {time.perf_counter() - t0:.1f}s")

    cpu = None
    one_core = None
    if not args.no_cpu:
        cores = max(1, min(16, os.cpu_count() or 1))
        sample = min(args.cpu_sample, n)
        cpu = cpu_baseline(frames, ref, w.u, sample, cores)
        log(f"[bench] oracle: {sample} frames in {cpu['wall']:.1f}s wall on {cpu['cores']} cores "
            f"({cpu['cpu_s']:.1f}s CPU)")
        one_core = cpu_one_core(frames, ref, w.u, min(64, n))
        log(f"[bench] oracle on one core: {len(one_core[0])} frames in {one_core[1]:.1f}s")

    import torch

    from paper_2310_08770_amd import Tracker, decode

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calib_mib:
        a = torch.ones(args.copy_calib_mib * (1 << 18), dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
        log(f"[bench] copy calibration: {args.copy_calib_mib} MiB read + written")
    frames_t = torch.from_numpy(frames).to(dev)
    ref_t = torch.from_numpy(ref).to(dev)
    M = int(np.ceil(1.5 * w.u - 1e-9))

    # ---- batched, headline precision: the timed steps (no per-kernel events)
    tr = Tracker(upsample=w.u, precision=args.precision, streams=args.streams)
    tr.set_reference(ref_t)
    if args.chunk > 0:
        tr.set_chunk(N, args.chunk)
    chunk = tr.chunk(N) if (args.no_tune or args.chunk > 0) else tr.autotune(N, n)
    how = "pinned" if args.chunk > 0 else ("default" if args.no_tune else "autotuned")
    log(f"[bench] chunk {chunk} frames per launch ({how})")
    rois = tr.rois(frames_t)
    out = torch.empty((n, 72), dtype=torch.uint8, device=dev)
    total, lat = time_batched(tr, frames_t, rois, out, args.steps, args.warmup, torch)
    res = decode(out)
    value = n * args.steps / total
    log(f"[bench] batched {args.precision} ({args.streams} stream{'s' if args.streams > 1 else ''}): "
        f"{value:,.0f} frames/s, step p50 {np.median(lat)*1e3:.2f} ms")
    clocks = gpu_clocks()  # right after the timed steps, while the clocks are still up
    log(f"[bench] clocks {clocks}")
    tr.close()

    # ---- the same launches, each bracketed by HIP events on the call's stream:
    # per-stage device times and the dominant kernel's average launch duration
    prof_steps = max(3, min(args.steps, 10))
    trp = Tracker(upsample=w.u, precision=args.precision, profile=True)
    trp.set_reference(ref_t)
    trp.set_chunk(N, chunk)
    ptotal, _ = time_batched(trp, frames_t, trp.rois(frames_t), out, prof_steps, 1, torch)
    stages = trp.stage_times(reset=True)
    trp.close()
    stage_ms = {k: v[0] / prof_steps for k, v in stages.items() if v[1]}
    upd_ms, upd_launches = stages["updft"]
    per_launch_ms = upd_ms / max(1, upd_launches)
    frames_per_launch = n * prof_steps / max(1, upd_launches)
    flops_launch = updft_flops_per_frame(N, M, args.precision) * frames_per_launch
    achieved = flops_launch / (per_launch_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    kernel_tag = "k_updft_" + {"fp32": "f32", "bf16x2": "bf16x2_t256", "fp16x2": "fp16x2_t256"}[args.precision]
    kernel_tag += f"<{N}>"
    traffic_pf = measured_traffic(kernel_tag)
    roofline = {
        "kernel": kernel_tag,
        "bound": "mfma",
        "achieved": round(achieved, 2),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": None if traffic_pf is None else int(traffic_pf * frames_per_launch),
        "launch_ms": round(per_launch_ms, 4),
        "frames_per_launch": round(frames_per_launch, 1),
        "flops_per_frame": updft_flops_per_frame(N, M, args.precision),
        "timed": f"HIP events around each launch over {prof_steps} event-bracketed steps",
    }

    # ---- other legs
    legs = {}
    other = "bf16x2" if args.precision == "fp32" else "fp32"
    try:
        tr2 = Tracker(upsample=w.u, precision=other)
        tr2.set_reference(ref_t)
        if not args.no_tune and args.chunk == 0:
            tr2.autotune(N, n)
        out2 = torch.empty((n, 72), dtype=torch.uint8, device=dev)
        tot2, lat2 = time_batched(tr2, frames_t, tr2.rois(frames_t), out2, max(3, args.steps // 3), 2, torch)
        r2 = decode(out2)
        legs[f"batched_{other}"] = dict(frames_per_s=round(n * max(3, args.steps // 3) / tot2, 1),
                                        p50_ms=round(float(np.median(lat2)) * 1e3, 3),
                                        p99_ms=round(float(np.percentile(lat2, 99)) * 1e3, 3))
        tr2.close()
    except Exception as e:  # the other precision may not be available
        r2 = None
        legs[f"batched_{other}"] = dict(error=str(e)[:200])

    # the fp16 split (same kernels, fp16 hi + lo operands) at the headline chunk,
    # with its agreement with the headline results
    r5 = None
    if not args.no_extra and args.precision == "bf16x2":
        try:
            tr5 = Tracker(upsample=w.u, precision="fp16x2", streams=args.streams)
            tr5.set_reference(ref_t)
            tr5.set_chunk(N, chunk)
            out5 = torch.empty((n, 72), dtype=torch.uint8, device=dev)
            k5 = max(3, args.steps // 3)
            tot5, lat5 = time_batched(tr5, frames_t, tr5.rois(frames_t), out5, k5, 2, torch)
            r5 = decode(out5)
            legs["batched_fp16x2"] = dict(
                frames_per_s=round(n * k5 / tot5, 1), chunk=chunk,
                p50_ms=round(float(np.median(lat5)) * 1e3, 3),
                same_integer_peak=bool(np.array_equal(r5["p"], res["p"])),
                max_dd_vs_bf16x2_px=float(np.max(np.abs(r5["d"] - res["d"]))))
            log(f"[bench] fp16x2: {n * k5 / tot5:,.0f} frames/s, {legs['batched_fp16x2']}")
            tr5.close()
        except Exception as e:  # noqa: BLE001
            legs["batched_fp16x2"] = dict(error=str(e)[:200])

    # the headline precision on the other stream setting (one stream: every launch
    # after the previous one; two: alternate chunks on two streams, the DFT of one
    # chunk overlapping the FFTs of the next); results are bit-identical
    other_streams = 3 - args.streams
    sname = "one_stream" if other_streams == 1 else "two_streams"
    if not args.no_extra:
        try:
            tr3 = Tracker(upsample=w.u, precision=args.precision, streams=other_streams)
            tr3.set_reference(ref_t)
            if args.chunk > 0:
                tr3.set_chunk(N, args.chunk)
            chunk3 = tr3.chunk(N) if (args.no_tune or args.chunk > 0) else tr3.autotune(N, n)
            out3 = torch.empty((n, 72), dtype=torch.uint8, device=dev)
            k3 = max(3, args.steps // 3)
            tot3, lat3 = time_batched(tr3, frames_t, tr3.rois(frames_t), out3, k3, 2, torch)
            legs[f"batched_{args.precision}_{sname}"] = dict(
                frames_per_s=round(n * k3 / tot3, 1), chunk=chunk3,
                p50_ms=round(float(np.median(lat3)) * 1e3, 3),
                bit_identical=bool(torch.equal(out3, out)))
            log(f"[bench] {sname.replace('_', ' ')}: {n * k3 / tot3:,.0f} frames/s (chunk {chunk3})")
            tr3.close()
        except Exception as e:  # noqa: BLE001
            legs[f"batched_{args.precision}_{sname}"] = dict(error=str(e)[:200])

    # the headline precision with the launch plan the autotuner picks on this machine
    if not args.no_extra and not args.no_tune and args.chunk > 0:
        try:
            tr4 = Tracker(upsample=w.u, precision=args.precision, streams=args.streams)
            tr4.set_reference(ref_t)
            chunk4 = tr4.autotune(N, n)
            k4 = max(3, args.steps // 3)
            tot4, lat4 = time_batched(tr4, frames_t, tr4.rois(frames_t), out, k4, 2, torch)
            legs[f"batched_{args.precision}_autotuned"] = dict(
                frames_per_s=round(n * k4 / tot4, 1), plan=tr4.plan(N),
                p50_ms=round(float(np.median(lat4)) * 1e3, 3))
            log(f"[bench] autotuned: {n * k4 / tot4:,.0f} frames/s (plan {tr4.plan(N)})")
            tr4.close()
        except Exception as e:  # noqa: BLE001
            legs[f"batched_{args.precision}_autotuned"] = dict(error=str(e)[:200])

    if not args.no_plain:
        for name, graph in (("plain", False), ("graph_stream", True)):
            trp = Tracker(upsample=w.u, precision="fp32", graph=graph)
            trp.set_reference(ref_t)
            time_plain(trp, frames_t, 50, torch)  # warm-up (captures the graph)
            lp = time_plain(trp, frames_t, args.plain_frames, torch)
            legs[name] = dict(frames_per_s=round(len(lp) / lp.sum(), 1),
                              p50_ms=round(float(np.median(lp)) * 1e3, 4),
                              p99_ms=round(float(np.percentile(lp, 99)) * 1e3, 4),
                              frames=len(lp))
            log(f"[bench] {name}: p50 {legs[name]['p50_ms']:.3f} ms p99 {legs[name]['p99_ms']:.3f} ms")
            trp.close()
        # the real-time path of Sec. III.B: each call tracks one frame and
        # low-pass updates the reference (Eq. 9), a0 = 0.01; at 256x256, u = 100
        # and at the paper's own real-time setting, 256x128 at u = 256 (Sec. IV.A)
        w_rt = S.table1_frames(256, 128, min(args.plain_frames, 512) + 50)
        rt_rect = torch.from_numpy(np.stack(w_rt.frames)).to(dev)
        for mode, fr_rt, u_rt, tag in (("ccu", frames_t, w.u, ""), ("ccsn", frames_t, w.u, ""),
                                       ("ccu", rt_rect, 256, "_256x128_u256"),
                                       ("ccsn", rt_rect, 256, "_256x128_u256")):
            name = f"realtime_{mode}{tag}"
            try:
                trr = Tracker(upsample=u_rt, precision="fp32", mode=mode)
                trr.set_reference(fr_rt[0].to(torch.float32))
                one = torch.empty((1, 72), dtype=torch.uint8, device=dev)
                nf = fr_rt.shape[0]
                lr = []
                for i in range(min(args.plain_frames, nf - 50) + 50):
                    t0 = time.perf_counter()
                    trr.track_update(fr_rt[i % nf], 0.01, out=one)
                    torch.cuda.synchronize()
                    lr.append(time.perf_counter() - t0)
                lr = np.array(lr[50:])
                legs[name] = dict(frames_per_s=round(len(lr) / lr.sum(), 1),
                                  p50_ms=round(float(np.median(lr)) * 1e3, 4),
                                  p99_ms=round(float(np.percentile(lr, 99)) * 1e3, 4), frames=len(lr))
                if tag:
                    legs[name]["paper_camera_rate_images_per_s"] = 470
                log(f"[bench] {name}: p50 {legs[name]['p50_ms']:.3f} ms p99 {legs[name]['p99_ms']:.3f} ms")
                trr.close()
            except Exception as e:  # noqa: BLE001
                legs[name] = dict(error=str(e)[:200])
        # where a plain call spends its GPU time
        trp = Tracker(upsample=w.u, precision="fp32", profile=True)
        trp.set_reference(ref_t)
        time_plain(trp, frames_t, 20, torch)
        trp.stage_times(reset=True)
        time_plain(trp, frames_t, 200, torch)
        st = trp.stage_times(reset=True)
        legs["plain"]["gpu_stage_us"] = {k: round(v[0] / max(1, v[1]) * 1e3, 2) for k, v in st.items() if v[1]}
        trp.close()

    # ---- the other workloads (each guarded: a failure is recorded, not fatal)
    if not args.no_extra:
        for name, fn in (("uneven_rois_u100", leg_uneven_rois), ("gauss512_u200", leg_gauss512),
                         ("gauss128_grad", leg_grad128), ("table1_ccsn", leg_table1),
                         ("fig1_w32", leg_fig1)):
            t0 = time.perf_counter()
            try:
                legs[name] = fn(dev, torch, Tracker)
            except Exception as e:  # noqa: BLE001
                legs[name] = dict(error=str(e)[:300])
            log(f"[bench] {name}: {legs[name]} ({time.perf_counter() - t0:.1f} s)")

    # ---- accuracy against the oracle sample
    accuracy = None
    cpu_json = None
    if cpu is not None:
        k = len(cpu["d"])
        ok = (cpu["status"] & (4 | 8 | 16)) == 0
        err = np.max(np.abs(res["d"][:k] - cpu["d"]), axis=1)
        peaks_equal = np.all(res["p"][:k] == cpu["p"], axis=1)

        def grid_stats(r, prec):
            # the grid estimate (the paper's sub-pixel result) against the
            # oracle's: same grid point on every frame, and on the frames whose
            # oracle top-two grid values differ by more than the precision's
            # rounding (2^-20 of the grid maximum's AC part in FP32, 2^-17 with
            # bf16 hi + lo operands, 2^-18 with fp16 hi + lo; the rest are
            # decided by rounding)
            same = np.max(np.abs(r["d_grid"][:k].astype(np.float64) - cpu["d_grid"]), axis=1) < 0.5 / w.u
            tol = {"fp32": 2.0 ** -20, "fp16x2": 2.0 ** -18}.get(prec, 2.0 ** -17)
            firm = cpu["grid_gap"] > tol * cpu["grid_ac"]
            gerr = np.max(np.abs(r["d_grid"][:k].astype(np.float64) - cpu["d_grid"]), axis=1)
            return dict(grid_index_agreement=float(same.mean()),
                        grid_index_agreement_beyond_rounding=float(same[firm].mean()) if firm.any() else None,
                        frames_beyond_rounding=int(firm.sum()),
                        max_grid_err_px=float(gerr.max()), p99_grid_err_px=float(np.percentile(gerr, 99)))

        accuracy = dict(frames_checked=int(k), max_err_px=float(err[ok].max()),
                        p99_err_px=float(np.percentile(err[ok], 99)),
                        mean_err_px=float(err[ok].mean()), integer_peak_agreement=float(peaks_equal.mean()),
                        oracle_fallbacks=int((~ok).sum()), oracle_near_ties=int(((cpu["status"] & 4) != 0).sum()),
                        **grid_stats(res, args.precision))
        if r2 is not None:
            e2 = np.max(np.abs(r2["d"][:k] - cpu["d"]), axis=1)
            accuracy[other] = dict(max_err_px=float(e2[ok].max()), p99_err_px=float(np.percentile(e2[ok], 99)),
                                   **grid_stats(r2, other))
        if r5 is not None:
            e5 = np.max(np.abs(r5["d"][:k] - cpu["d"]), axis=1)
            accuracy["fp16x2"] = dict(max_err_px=float(e5[ok].max()), p99_err_px=float(np.percentile(e5[ok], 99)),
                                      **grid_stats(r5, "fp16x2"))
        cpu_json = {
            "value": round(k / cpu["wall"], 2),
            "unit": "frames/s",
            "cores": cpu["cores"],
            "kind": "oracle",
            "sample": f"first {k} of the {n} frames (256x256, u=100), FP64 numpy oracle, "
                      f"one single-threaded process per core; {cpu['cpu_s']:.1f} s of CPU work",
            "mean_ms_per_frame_per_core": round(1e3 * cpu["cpu_s"] / k, 3),
            "cpu": cpu_model(),
            "one_core": None if one_core is None else {
                "frames_per_s": round(len(one_core[0]) / one_core[1], 2),
                "p50_ms_per_frame": round(float(np.median(one_core[0])) * 1e3, 3),
                "p99_ms_per_frame": round(float(np.percentile(one_core[0], 99)) * 1e3, 3),
                "sample": f"first {len(one_core[0])} frames, one single-threaded process"},
        }

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": f"airy256_u100: {n} frames of {N}x{N} uint16 (12-bit) Airy spots, random walk, "
                        f"u=100, 1.5-px window (M={M}), CC-U, {args.precision} upsampled DFT, FP64 Newton x3",
            "frames_per_step": n,
            "upsample": w.u,
            "chunk": chunk,
            "streams": args.streams,
        },
        "batched_latency": {"p50_ms": round(float(np.median(lat)) * 1e3, 4),
                            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4)},
        "stage_ms_per_step": {k: round(v, 4) for k, v in stage_ms.items()},
        "profiled_ms_per_step": round(ptotal / prof_steps * 1e3, 4),
        "legs": legs,
        "roofline": roofline,
        "cpu_baseline": cpu_json,
        "accuracy": accuracy,
        "hbm_bytes_per_frame": int(N * N * 2),
        "gpu_clocks": clocks,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
