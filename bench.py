"""Benchmark: LED-tile updates per second of the full reconstruction.

Workload (default): the full field of view of a 2048 x 2048 sensor cut into
16 x 16 overlapping tiles of 128 px (8 px overlap), each with its own
illumination angles (tile position) and defocus z ~ U[-20, 20] um, 15 x 15
LEDs (4 mm pitch, 90 mm high), 4x upsampling (512 x 512 spectrum per tile),
20 iterations, LED groups run concurrently (spectrum-domain parallel form),
pupil recovery on, FP32 FFT path.  One step = one complete reconstruction
of all 256 tiles = 256 * 225 * 20 = 1,152,000 LED-tile updates, with the
intensity stack already resident in HBM.

Inputs are synthetic and seeded (fpm_synth): per-tile objects, the forward
model run by the library itself, Poisson noise at 1e4 peak photons drawn
with a seeded torch generator on the device.  Parity of this configuration
with the FP64 oracle is checked by the GPU tests; here the oracle only runs
as the CPU baseline.

Prints one JSON line (rank 0): metric, value, roofline of the update kernel
(HIP events per launch), the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, vendor figure
MFMA_PEAK_TFLOPS = 2500.0    # MI355X dense bf16 / fp16 matrix peak, vendor figure
PREC_NAMES = {1: "mfma_bf16x3", 2: "mfma_fp16"}
PREC_TERMS = {1: 3, 2: 1}    # real MFMA products per real product
KERNEL_SRC = os.path.join(ROOT, "paper_2203_02507_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "update_kernel_128_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def make_inputs(fpm, tds, device):
    """Objects (numpy, seeded) -> library forward model -> Poisson noise."""
    import numpy as np
    import torch
    import fpm_synth

    descs = []
    objs = []
    for td in tds:
        objs.append(fpm_synth.draw_object_and_defocus(td, 20.0).astype(np.complex64))
        descs.append(td.desc)
    plan = fpm.Plan(descs)
    o = torch.from_numpy(np.concatenate([x.reshape(-1) for x in objs]).view(np.float32)).to(device)
    del objs
    I = torch.empty(plan.total_intensity, dtype=torch.float32, device=device)
    fpm.fpm_forward(plan, o, None, I, fpm.FPM_MEM_DEVICE)
    torch.cuda.synchronize()
    del o
    gen = torch.Generator(device=device)
    gen.manual_seed(fpm_synth.ROOT_SEED)
    for t, info in enumerate(plan.infos):
        sl = I[info.intensity_offset:info.intensity_offset + info.L * info.n * info.n]
        c = tds[t].peak_photons / float(sl.max())
        sl.copy_(torch.poisson(sl.clamp_min(0) * c, generator=gen) / c)
    torch.cuda.synchronize()
    return plan, I


def roofline(plan, prof):
    """Algorithmic HBM bytes of the update kernel per unit of its run time.

    Per LED-tile update: read the intensity image (4 n^2 B), read and write
    the support pixels of the spectrum window (2 * 8 |D0| B).  The chains of
    tiles overlap their launches, so a launch's duration is not its cost:
    achieved = algorithmic bytes of all update launches / the time at least
    one of them ran (the union of their intervals, HIP events); with one
    chain this is bytes per launch / mean launch duration."""
    upd = prof["update"]
    info = plan.infos[0]
    b_upd = 4 * info.n * info.n + 16 * info.support_count
    per_launch_items = upd["items"] / max(upd["launches"], 1)
    mean_s = upd["total_ms"] / 1e3 / max(upd["launches"], 1)
    busy_s = upd["busy_ms"] / 1e3
    achieved = b_upd * upd["items"] / busy_s / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        if rec.get("kernel_sha256_16") == kernel_hash():
            traffic = rec.get("hbm_bytes_per_launch")
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"update_kernel<{info.n}>", "bytes_per_update": b_upd,
            "updates_per_launch": round(per_launch_items, 1),
            "launches": upd["launches"], "busy_ms": round(upd["busy_ms"], 3),
            "mean_launch_us": round(mean_s * 1e6, 2),
            "bytes_per_launch": round(b_upd * per_launch_items, 1)}


def mfma_flops_per_update(desc, prec):
    """Matrix-core FLOPs one update issues in the MFMA kernel: 32x32x16 tile
    steps of the four products (E Phi^T, E M1^T, F psi', F V^T) over the
    support box, 4 real products per complex step, `terms` per real product."""
    n = desc.n
    R = math.floor(desc.na_obj * n * desc.pixel_um / desc.wavelength_um)
    kx0, nd = n // 2 - R, 2 * R + 1
    ub = kx0 & ~7
    nk = (kx0 + nd - ub + 15) // 16
    mt = (16 * nk + 31) // 32
    W, KS = n // 32, n // 16
    steps = W * nk * mt + W * nk * W + W * mt * KS + mt * mt * KS
    dense = 16 * n * nd * (n + nd)   # unpadded complex DFT products on the support
    return steps * 4 * 2 * 32 * 32 * 16 * PREC_TERMS[prec], dense * PREC_TERMS[prec]


def host_cpu():
    """The host the oracle runs on: logical CPUs, those this process may use,
    and the CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count() or 1, "usable": usable, "model": model}


def rel_l2(a, b) -> float:
    import numpy as np
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / nb if nb > 0 else float(np.linalg.norm(a))


def small_uneven_tiles(fpm, count: int, max_updates: int = 2500):
    """The first `count` tiles of the uneven workload's draw (n <= 128, at
    most `max_updates` updates each) whose geometry the library accepts."""
    import fpm_synth
    out = []
    for td in fpm_synth.uneven_batch(T=512, sizes=(64, 96, 128, 256)):
        d = td.desc
        if d.n > 128 or d.led_rows * d.led_cols * d.iterations > max_updates:
            continue
        if pick_upsample(fpm, td):
            out.append(td)
        if len(out) == count:
            break
    return out


def cpu_baseline(fpm, n_tiles: int = 16, threads_cap: int = 16):
    """The FP64 oracle timed on a bounded sample of the benchmark's workload:
    the first `n_tiles` full-field tiles for all their iterations, one tile
    per host thread (the usable host CPUs, at most `threads_cap`: the host
    share of one GPU).  Its results are also the reference for the accuracy
    of every GPU form reported beside the throughput, computed here, outside
    every timed region, on the same seeded stacks (the oracle's forward model
    with shot noise): the FP32 path and each MFMA precision on these tiles,
    two small tiles of the uneven workload run as one batched plan, and two
    requests (FP32 and BF16x3) through the server."""
    from concurrent.futures import ThreadPoolExecutor
    import dataclasses
    import numpy as np
    import torch
    import fpm_synth
    import oracle

    host = host_cpu()
    threads = max(1, min(n_tiles, host["usable"], threads_cap))
    oracle.set_threads(1)
    tds = fpm_synth.full_fov_tiles(only=list(range(n_tiles)))
    with ThreadPoolExecutor(threads) as ex:
        stacks = list(ex.map(lambda td: oracle.synthesize(td, z_range=20.0)[2], tds))
    descs = [td.desc for td in tds]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda a: oracle.reconstruct(a[0], a[1]), zip(descs, stacks)))
    wall = time.perf_counter() - t0
    assert all(r.status == 0 for r in res)
    updates = sum(d.led_rows * d.led_cols * d.iterations for d in descs)
    refs = [(oracle.spectrum_to_object(d, r.S), r.P) for d, r in zip(descs, res)]
    log(f"cpu baseline: {updates} oracle updates in {wall:.1f} s on {threads} threads")

    def gpu_run(ds, Is):
        plan = fpm.Plan(ds)
        I = torch.from_numpy(np.concatenate([x.reshape(-1) for x in Is])).cuda()
        obj, pup, res_d = fpm.device_buffers(plan)
        fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj, pup, res_d)
        torch.cuda.synchronize()
        return fpm.split_tiles(plan, obj.cpu().numpy(), pup.cpu().numpy(), res_d.cpu().numpy())

    acc = {}
    for prec, name in ((0, "fp32_fft"), (1, "mfma_bf16x3"), (2, "mfma_fp16")):
        out = gpu_run([dataclasses.replace(d, precision=prec) for d in descs], stacks)
        eo = [rel_l2(o, r[0]) for (o, _, _), r in zip(out, refs)]
        ep = [rel_l2(p, r[1]) for (_, p, _), r in zip(out, refs)]
        acc[name] = {"tiles": n_tiles, "object_max": float(f"{max(eo):.3e}"),
                     "object_mean": float(f"{sum(eo) / len(eo):.3e}"),
                     "pupil_max": float(f"{max(ep):.3e}"),
                     "tolerance": 1e-4 if prec == 0 else 1e-3}

    # uneven workload (batched plan) and served requests, small samples
    small = small_uneven_tiles(fpm, 4)
    ud = [td.desc for td in small[:2]]
    uI = [oracle.synthesize(td)[2] for td in small[:2]]
    sd = [dataclasses.replace(small[2].desc, precision=0),
          dataclasses.replace(small[3].desc, precision=1)]
    sI = [oracle.synthesize(td)[2] for td in small[2:4]]
    with ThreadPoolExecutor(4) as ex:
        r_all = list(ex.map(lambda a: oracle.reconstruct(a[0], a[1]), zip(ud + sd, uI + sI)))
    ref_all = [oracle.spectrum_to_object(d, r.S) for d, r in zip(ud + sd, r_all)]
    out_u = gpu_run(ud, uI)
    acc["uneven_batch"] = {
        "tiles": [f"n={d.n} {d.led_rows}x{d.led_cols} LEDs {d.iterations} it" for d in ud],
        "object": [float(f"{rel_l2(o[0], r):.3e}") for o, r in zip(out_u, ref_all[:2])],
        "tolerance": 1e-4}
    srv = fpm.Server(1 << 30, max_slots=8)
    ids = [srv.submit(d, torch.from_numpy(I.reshape(-1)).cuda(), fpm.FPM_MEM_DEVICE)
           for d, I in zip(sd, sI)]
    served = [srv.wait(i, d)[0] for i, d in zip(ids, sd)]
    srv.close()
    acc["serving"] = {
        "requests": [f"n={d.n} {d.led_rows}x{d.led_cols} LEDs {d.iterations} it "
                     f"{'fp32_fft' if d.precision == 0 else 'mfma_bf16x3'}" for d in sd],
        "object": [float(f"{rel_l2(o[0], r):.3e}") for o, r in zip(served, ref_all[2:])],
        "tolerance": [1e-4, 1e-3]}
    baseline = {"value": round(updates / wall, 2), "unit": "updates/s", "cores": threads,
                "kind": "oracle",
                "sample": f"{n_tiles} tiles x {descs[0].iterations} iterations x 225 LEDs of "
                          f"the 128-px full-field workload ({updates} updates, {wall:.1f} s "
                          f"wall), one tile per thread",
                "host": host}
    return baseline, acc


def pick_upsample(fpm, td):
    d = td.desc
    for up in td.up_candidates:
        d.upsample = up
        try:
            fpm.Plan([d])
            return True
        except fpm.FpmError:
            pass
    return False


def single_tile_bench(fpm, reps: int = 5):
    """One 64-px tile, 15x15 LEDs, 10 iterations (2,250 updates), LEDs in
    ascending illumination NA: the latency of one reconstruction for the
    sequential sweep (pupil recovery on and off) and for the pipelined
    schedule (Sec. 3.2 Fig. 6b/d, level-scheduled over iterations; the same
    bits as sequential), mean over `reps` runs."""
    import numpy as np
    import torch
    import fpm_synth

    out = {}
    td = fpm_synth.single_tile_64()[0]
    obj = fpm_synth.draw_object_and_defocus(td, None).astype(np.complex64)
    for name, sched, pupil in (("sequential_pupil", 0, 1), ("sequential", 0, 0),
                               ("pipelined", 3, 0), ("led_groups", 1, 0)):
        d = fpm_synth.single_tile_64(schedule=sched, pupil_update=pupil)[0].desc
        plan = fpm.Plan([d])
        o = torch.from_numpy(obj.reshape(-1).view(np.float32)).cuda()
        I = torch.empty(plan.total_intensity, dtype=torch.float32, device="cuda")
        fpm.fpm_forward(plan, o, None, I, fpm.FPM_MEM_DEVICE)
        ob, pu, re = fpm.device_buffers(plan)
        fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, ob, pu, re)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, ob, pu, re)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        info = plan.infos[0]
        out[name] = {"ms": round(ms, 3), "dependent_launches": info.levels,
                     "updates_per_s": round(info.L * info.iterations / (ms / 1e3), 1)}
    out["pipelined_speedup_vs_sequential"] = round(out["sequential"]["ms"] / out["pipelined"]["ms"], 2)
    return out


def online_bench(fpm, tds, I, tiles_per_side: int, counts=(16, 256)):
    """Online strategy (Sec. 3.4 Fig. 7a): the full-field tiles with the
    sequential schedule, one LED's images of every tile pushed at a time (in
    NA order, from device memory), each push running that LED's update on
    all tiles; after the last push fpm_online_finish runs the remaining
    iterations.  Per count of tiles (the centre block of the field): GPU time
    per push (HIP events around each push, synchronised), the host time of a
    push call, and the finish time."""
    import dataclasses
    import statistics
    import torch

    out = {}
    n = tds[0].desc.n
    L = tds[0].desc.led_rows * tds[0].desc.led_cols
    Iv = I.view(len(tds), L, n * n)
    for T in counts:
        side = int(round(T ** 0.5))
        if side * side != T or side > tiles_per_side:
            continue
        lo = (tiles_per_side - side) // 2
        idx = [(lo + r) * tiles_per_side + lo + c for r in range(side) for c in range(side)]
        descs = [dataclasses.replace(tds[t].desc, schedule=fpm.FPM_SCHED_SEQUENTIAL) for t in idx]
        plan = fpm.Plan(descs)
        order = plan.tables(0)[1]
        imgs = Iv[idx].transpose(0, 1).contiguous()  # [L][tile][n*n]
        obj, pup, res = fpm.device_buffers(plan)
        fpm.fpm_online_begin(plan)  # setup and tuning outside the timing
        for j in order:
            fpm.fpm_online_push(plan, int(j), imgs[int(j)], fpm.FPM_MEM_DEVICE)
        fpm.fpm_online_finish(plan, fpm.FPM_MEM_DEVICE, obj, pup, res)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        gpu_ms, host_ms = [], []
        fpm.fpm_online_begin(plan)
        for j in order:
            torch.cuda.synchronize()
            e0.record()
            h0 = time.perf_counter()
            fpm.fpm_online_push(plan, int(j), imgs[int(j)], fpm.FPM_MEM_DEVICE)
            host_ms.append((time.perf_counter() - h0) * 1e3)
            e1.record()
            torch.cuda.synchronize()
            gpu_ms.append(e0.elapsed_time(e1))
        f0 = time.perf_counter()
        fpm.fpm_online_finish(plan, fpm.FPM_MEM_DEVICE, obj, pup, res)
        torch.cuda.synchronize()
        fin_ms = (time.perf_counter() - f0) * 1e3
        out[f"{T}_tiles"] = {
            "tiles": T, "leds": L, "iterations": descs[0].iterations,
            "push_gpu_ms_mean": round(statistics.mean(gpu_ms), 4),
            "push_gpu_ms_median": round(statistics.median(gpu_ms), 4),
            "push_gpu_ms_max": round(max(gpu_ms), 4),
            "push_host_ms_median": round(statistics.median(host_ms), 4),
            "first_iteration_gpu_ms": round(sum(gpu_ms), 3),
            "finish_ms": round(fin_ms, 3),
            "updates_per_push": T,
        }
        del plan, imgs, obj, pup, res
    return out


def host_mode_bench(fpm, plan, I, updates):
    """fpm_reconstruct with host buffers: the intensity stack (pageable numpy)
    validated by host threads into pinned chunks whose uploads overlap the
    checking, the reconstruction, and the object, pupil and residuals copied
    back -- the rate a caller holding its data in host memory sees (PCIe
    included).  One run after a warm-up."""
    import numpy as np
    Ih = I.cpu().numpy()
    obj = np.empty(plan.total_object * 2, np.float32)
    pup = np.empty(plan.total_pupil * 2, np.float32)
    res = np.empty(max(plan.total_residual, 1), np.float64)
    fpm.fpm_reconstruct(plan, Ih, fpm.FPM_MEM_HOST, obj, pup, res)
    t0 = time.perf_counter()
    fpm.fpm_reconstruct(plan, Ih, fpm.FPM_MEM_HOST, obj, pup, res)
    s = time.perf_counter() - t0
    return {"ms": round(s * 1e3, 1), "updates_per_s": round(updates / s, 1),
            "intensity_gib": round(Ih.nbytes / 2**30, 2),
            "note": "threaded host validation into pinned chunks + overlapped H2D of the stack + "
                    "reconstruction + D2H of object, pupil and residuals; not the benchmark value"}


def paper_workload_bench(fpm, reps: int = 3):
    """The paper's own GPU timing workload, as context: 169 LR images (13 x 13
    LEDs, 2.5 mm pitch, 83 mm high, NA 0.1, 2.4 um camera pixels behind a 2x
    objective), 16 sub-regions of 256 x 256 px (26 px overlap), one iteration.
    The paper does not state the wavelength or the upsampling: 0.532 um and 4x
    here.  Synthetic seeded objects and defocus, library forward model,
    Poisson noise; sequential NA-order sweep and LED groups, mean of `reps`
    runs (HIP events)."""
    import numpy as np
    import torch
    import fpm_synth

    rng = np.random.default_rng(2203)
    stride, pix = 256 - 26, 1.2
    descs = []
    for ty in range(4):
        for tx in range(4):
            descs.append(fpm_synth.TileDesc(
                n=256, upsample=4, led_rows=13, led_cols=13, led_pitch_um=2500.0,
                led_height_um=83000.0, pixel_um=pix, na_obj=0.1, iterations=1,
                tile_x_um=(tx - 1.5) * stride * pix, tile_y_um=(ty - 1.5) * stride * pix,
                defocus_um=float(rng.uniform(-20, 20))))
    out = {}
    for name, sched in (("sequential", fpm.FPM_SCHED_SEQUENTIAL),
                        ("led_groups", fpm.FPM_SCHED_LED_GROUPS)):
        for d in descs:
            d.schedule = sched
        plan = fpm.Plan(descs)
        objs = [fpm_synth.random_object(rng, d.N).astype(np.complex64) for d in descs]
        o = torch.from_numpy(np.concatenate([x.reshape(-1) for x in objs]).view(np.float32)).cuda()
        I = torch.empty(plan.total_intensity, dtype=torch.float32, device="cuda")
        fpm.fpm_forward(plan, o, None, I, fpm.FPM_MEM_DEVICE)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(fpm_synth.ROOT_SEED)
        I = torch.poisson(I.clamp_min(0) * (1e4 / float(I.max())), generator=gen) * (
            float(I.max()) / 1e4)
        ob, pu, re = fpm.device_buffers(plan)
        fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, ob, pu, re)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, ob, pu, re)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": round(ms, 3), "updates": 16 * 169,
                     "updates_per_s": round(16 * 169 / (ms / 1e3), 1)}
        del plan, o, I, ob, pu, re
    out["paper_gpu_context"] = ("GTX 1050 laptop GPU, PyTorch: about 1.0 s for one sub-region "
                                "and 0.9 s per further one (Sec. 4.1), i.e. about 14.5 s for 16; "
                                "0.1 s per LR image for 16 sub-regions online (Sec. 3.4)")
    return out


def uneven_objects(tds, device):
    """Seeded objects of every tile (host threads), packed on the device."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import torch
    import fpm_synth

    total = sum(td.desc.N ** 2 for td in tds)
    o = torch.empty(2 * total, dtype=torch.float32, device=device)
    offs, acc = [], 0
    for td in tds:
        offs.append(acc)
        acc += td.desc.N ** 2

    def one(k):
        td = tds[k]
        return k, fpm_synth.random_object(td.rng, td.desc.N).astype(np.complex64)

    with ThreadPoolExecutor(16) as ex:
        for k, obj in ex.map(one, range(len(tds))):
            sl = o[2 * offs[k]:2 * (offs[k] + tds[k].desc.N ** 2)]
            sl.copy_(torch.from_numpy(obj.reshape(-1).view(np.float32)))
    return o


def uneven_bench(fpm, T: int, steps: int, warmup: int, sample: int = 16):
    """Batched form: T uneven tiles (n in {64, 96, 128, 256}, 9x9..21x21 LEDs,
    upsampling 3-5, 5-30 iterations, defocus, 1e3-1e5 photons) in one plan,
    one launch per (size, step) over all tiles, replayed from a graph.  Beside
    it, the first `sample` tiles run one plan per tile (no batching across
    tiles) and as one plan, so the batching gain is measured on equal work."""
    import torch
    import fpm_synth

    device = "cuda"
    t0 = time.perf_counter()
    tds = [td for td in fpm_synth.uneven_batch(T=T, sizes=(64, 96, 128, 256))
           if pick_upsample(fpm, td)]
    plan = fpm.Plan([td.desc for td in tds])
    o = uneven_objects(tds, device)
    I = torch.empty(plan.total_intensity, dtype=torch.float32, device=device)
    fpm.fpm_forward(plan, o, None, I, fpm.FPM_MEM_DEVICE)
    gen = torch.Generator(device=device)
    gen.manual_seed(fpm_synth.ROOT_SEED + 3)
    for t, info in enumerate(plan.infos):
        sl = I[info.intensity_offset:info.intensity_offset + info.L * info.n * info.n]
        c = tds[t].peak_photons / max(float(sl.max()), 1e-30)
        sl.copy_(torch.poisson(sl.clamp_min(0) * c, generator=gen) / c)
    del o
    torch.cuda.synchronize()
    log(f"uneven inputs: {len(tds)} tiles, {I.numel() * 4 / 2**30:.2f} GiB in "
        f"{time.perf_counter() - t0:.1f} s")
    obj, pup, res = fpm.device_buffers(plan, device)
    updates = sum(i.L * i.iterations for i in plan.infos)

    def timed(pl, Iv, k):
        for _ in range(warmup):
            fpm.fpm_reconstruct(pl, Iv, fpm.FPM_MEM_DEVICE, obj, pup, res)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fpm.fpm_reconstruct(pl, Iv, fpm.FPM_MEM_DEVICE, obj, pup, res)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms = timed(plan, I, steps)
    r = res.cpu().numpy()
    if not all(math.isfinite(x) for x in r):
        raise SystemExit("uneven batch: non-finite residual")
    prof = fpm.fpm_profile_reconstruct(plan, I)
    torch.cuda.synchronize()
    # algorithmic HBM bytes of all update launches (per update: the intensity
    # image read, the spectrum support read and written) over the time at
    # least one update launch ran
    alg_bytes = sum(i.L * i.iterations * (4 * i.n * i.n + 16 * i.support_count)
                    for i in plan.infos)
    upd = prof["update"]
    achieved = alg_bytes / (upd["busy_ms"] / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "update kernels of every tile size", "algorithmic_bytes": alg_bytes,
            "busy_ms": round(upd["busy_ms"], 3),
            "frac_whole_step": round(alg_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    by_n = {}
    for i in plan.infos:
        b = by_n.setdefault(str(i.n), {"tiles": 0, "updates": 0})
        b["tiles"] += 1
        b["updates"] += i.L * i.iterations
    # batching gain on the first `sample` tiles
    ns = min(sample, len(tds))
    sub = fpm.Plan([td.desc for td in tds[:ns]])
    sub_I = torch.cat([I[i.intensity_offset:i.intensity_offset + i.L * i.n * i.n]
                       for i in plan.infos[:ns]])
    sub_updates = sum(i.L * i.iterations for i in plan.infos[:ns])
    ms_batched = timed(sub, sub_I, 1)
    ms_single = 0.0
    for k in range(ns):
        one = fpm.Plan([tds[k].desc])
        info = plan.infos[k]
        ms_single += timed(one, I[info.intensity_offset:info.intensity_offset +
                                  info.L * info.n * info.n], 1)
    return {"tiles": len(tds), "updates_per_step": updates, "ms_per_step": round(ms, 3),
            "value": round(updates / (ms / 1e3), 1), "unit": "updates/s", "by_n": by_n,
            "roofline": roof,
            "kernel_ms": {k: round(v["total_ms"], 3) for k, v in prof.items()},
            "update_launches": prof["update"]["launches"],
            "batching_gain": {"tiles": ns, "updates": sub_updates,
                              "one_plan_ms": round(ms_batched, 3),
                              "plan_per_tile_ms": round(ms_single, 3),
                              "speedup": round(ms_single / ms_batched, 2)}}


def serving_bench(fpm, pool: int = 96, warmup: int = 200, measured: int = 1000,
                  loads=(0.5, 0.8, 0.95), seed: int = 5):
    """Requests shaped like single uneven tiles (64-256 px, 9x9..21x21 LEDs,
    5..30 iterations; precision flags 50 % FP32, 25 % BF16x3, 25 % FP16 on
    the sizes the MFMA form runs), `pool` distinct ones cycled in a seeded
    order into `warmup` + `measured` submissions.  The saturated request rate
    comes from the measured part of a closed-loop run (all submitted at
    once); then, for each of `loads` x that rate, an open-loop Poisson
    stream of the same submissions: p50/p99 latency over the measured
    requests (the warm-up ones fill the server first and are not counted)
    and the sustained updates/s over them."""
    import numpy as np
    import torch
    import fpm_synth

    reqs = []
    mix_rng = np.random.default_rng(seed)
    for td in fpm_synth.uneven_batch(T=4 * pool, workload=4, sizes=(64, 96, 128, 256)):
        d = td.desc
        if d.n <= 128:
            d.precision = int(mix_rng.choice([0, 0, 1, 2]))
        for up in td.up_candidates:
            d.upsample = up
            try:
                plan = fpm.Plan([d])
                break
            except fpm.FpmError:
                plan = None
        if plan is None:
            continue
        obj = fpm_synth.random_object(td.rng, d.N).astype(np.complex64)
        o = torch.from_numpy(obj.reshape(-1).view(np.float32)).cuda()
        I = torch.empty(plan.total_intensity, dtype=torch.float32, device="cuda")
        fpm.fpm_forward(plan, o, None, I, fpm.FPM_MEM_DEVICE)
        torch.cuda.synchronize()
        c = td.peak_photons / float(I.max())
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed + len(reqs))
        I = torch.poisson(I.clamp_min(0) * c, generator=gen) / c
        reqs.append((d, I.contiguous()))
        if len(reqs) == pool:
            break
    torch.cuda.synchronize()
    total = warmup + measured
    order = np.random.default_rng(seed + 1).integers(0, len(reqs), size=total)
    seq = [reqs[k] for k in order]
    budget = int(0.5 * torch.cuda.mem_get_info()[0])
    srv = fpm.Server(budget, max_slots=256)

    def collect(ids):
        stats = [srv.wait(i, d)[1] for i, (d, _) in zip(ids, seq)]
        return stats[warmup:]

    # closed loop: everything at once -> saturated request rate
    ids = [srv.submit(d, I, fpm.FPM_MEM_DEVICE) for d, I in seq]
    st = collect(ids)
    first = min(x.submit_s for x in st)
    span = max(x.finish_s for x in st) - min(x.admit_s for x in st)
    sat_req = measured / span
    sat_updates = sum(x.updates for x in st) / span
    log(f"serving closed loop: {total} requests, {sat_req:.1f} requests/s, "
        f"{sat_updates / 1e6:.3f} M updates/s over the measured {measured}")
    by_load = {}
    for ld in loads:
        rate = ld * sat_req
        gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=total)
        start = time.perf_counter()
        due = start
        ids = []
        for (d, I), g in zip(seq, gaps):
            due += g
            while time.perf_counter() < due:
                time.sleep(min(1e-3, max(0.0, due - time.perf_counter())))
            ids.append(srv.submit(d, I, fpm.FPM_MEM_DEVICE))
        st = collect(ids)
        lat = np.array([x.finish_s - x.submit_s for x in st])
        first = min(x.submit_s for x in st)
        last = max(x.finish_s for x in st)
        by_load[str(ld)] = {
            "arrival_rate_per_s": round(rate, 2),
            "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "sustained_updates_per_s": round(sum(x.updates for x in st) / (last - first), 1)}
        log(f"serving load {ld}: " + json.dumps(by_load[str(ld)]))
    srv.close()
    return {"distinct_requests": len(reqs), "warmup_requests": warmup,
            "measured_requests": measured, "saturated_requests_per_s": round(sat_req, 2),
            "saturated_updates_per_s": round(sat_updates, 1), "by_load": by_load,
            "mix": "64-256 px tiles, 81-441 LEDs, 5-30 iterations, precision 50 % FP32, "
                   "25 % BF16x3, 25 % FP16 (FP32 for 256 px, which the MFMA form does not run)",
            "precisions": {str(p): int(sum(1 for d, _ in seq[warmup:] if d.precision == p))
                           for p in (0, 1, 2)},
            "budget_bytes": budget}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tiles-per-side", type=int, default=16)
    ap.add_argument("--iterations", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-online", action="store_true")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-tile latency section")
    ap.add_argument("--precisions", default="1,2",
                    help="MFMA precision variants timed beside the FP32 path (comma list, "
                         "empty for none)")
    ap.add_argument("--uneven-tiles", type=int, default=512,
                    help="tiles of the uneven batched workload (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (tiles are "
              "independent, so a multi-GPU run would shard tiles across GPUs).", file=sys.stderr)
        sys.exit(2)
    if args.no_graph:
        os.environ["FPM_NO_GRAPH"] = "1"

    import torch
    import fpm_synth
    import paper_2203_02507_amd as fpm

    device = "cuda:0"
    torch.cuda.set_device(0)
    tds = fpm_synth.full_fov_tiles(tiles_per_side=args.tiles_per_side, iterations=args.iterations,
                                   schedule=fpm.FPM_SCHED_LED_GROUPS, pupil_update=1)
    t0 = time.perf_counter()
    plan, I = make_inputs(fpm, tds, device)
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s: {len(tds)} tiles, "
        f"{I.numel() * 4 / 2**30:.2f} GiB of intensities on the device")
    obj, pup, res = fpm.device_buffers(plan, device)
    updates = sum(i.L * i.iterations for i in plan.infos)

    stream = torch.cuda.current_stream()
    for w in range(args.warmup):
        fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj, pup, res)
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj, pup, res)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    ms_per_step = ev_ms / args.steps
    value = updates * args.steps / (ev_ms / 1e3)
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step (events), wall {wall:.3f} s")
    r = res.cpu().numpy()
    if not all(math.isfinite(x) for x in r):
        raise SystemExit("non-finite residual")

    host_mode = None
    if not args.no_single:
        host_mode = host_mode_bench(fpm, plan, I, updates)
        log("host-buffer mode: " + json.dumps(host_mode))

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device=device).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    prof = fpm.fpm_profile_reconstruct(plan, I)
    torch.cuda.synchronize()
    log("kernel time per kind: " + json.dumps(prof))
    roof = roofline(plan, prof)

    stitch = None
    if args.tiles_per_side > 1:
        # Sec. 3.1 Eq. (1): the full field from the reconstructed tiles
        # (tile objects are row-major in plan order; 8 LR px overlap)
        ov = 8 * (plan.infos[0].N // plan.infos[0].n)
        R = args.tiles_per_side
        H, W = fpm.stitched_shape(R, R, plan.infos[0].N, ov)
        fov = torch.empty(2 * H * W, dtype=torch.float32, device=device)
        fpm.fpm_stitch(obj, R, R, plan.infos[0].N, ov, fov, fpm.FPM_MEM_DEVICE)
        t1 = time.perf_counter()
        for _ in range(3):
            fpm.fpm_stitch(obj, R, R, plan.infos[0].N, ov, fov, fpm.FPM_MEM_DEVICE)
        ms = (time.perf_counter() - t1) / 3 * 1e3
        moved = 2 * H * W * 8  # owned tile pixels read + result written
        stitch = {"tiles": f"{R}x{R}", "tile_side": plan.infos[0].N, "overlap": ov,
                  "out_shape": [H, W], "ms": round(ms, 3),
                  "gbs_algorithmic": round(moved / (ms / 1e3) / 1e9, 1),
                  "note": "wall time of fpm_stitch (returns after the result is written)"}
        del fov
        log("stitch: " + json.dumps(stitch))

    mfma = {}
    for prec in [int(x) for x in args.precisions.split(",") if x.strip()]:
        for td in tds:
            td.desc.precision = prec
        plan_p = fpm.Plan([td.desc for td in tds])
        for w in range(args.warmup):
            fpm.fpm_reconstruct(plan_p, I, fpm.FPM_MEM_DEVICE, obj, pup, res)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            fpm.fpm_reconstruct(plan_p, I, fpm.FPM_MEM_DEVICE, obj, pup, res)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        prof_p = fpm.fpm_profile_reconstruct(plan_p, I)
        torch.cuda.synchronize()
        upd = prof_p["update"]
        issued, dense = mfma_flops_per_update(tds[0].desc, prec)
        per_launch = upd["items"] / max(upd["launches"], 1)
        mean_s = upd["total_ms"] / 1e3 / max(upd["launches"], 1)
        achieved = issued * upd["items"] / (upd["busy_ms"] / 1e3) / 1e12
        mfma[PREC_NAMES[prec]] = {
            "value": round(updates / (ms / 1e3), 1), "unit": "updates/s",
            "ms_per_step": round(ms, 3),
            "vs_fp32": round(ms_per_step / ms, 3),
            "roofline": {"bound": "mfma", "achieved": round(achieved, 1),
                         "peak": MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(achieved / MFMA_PEAK_TFLOPS, 4), "traffic": None,
                         "kernel": f"mfma_update_kernel<{tds[0].desc.n}>",
                         "mfma_flops_per_update": issued,
                         "dense_dft_flops_per_update": dense,
                         # the same run time priced on the unpadded support's
                         # dense DFT products (no tile padding, no zero rows)
                         "frac_dense": round(dense * upd["items"] / (upd["busy_ms"] / 1e3)
                                             / 1e12 / MFMA_PEAK_TFLOPS, 4),
                         "updates_per_launch": round(per_launch, 1),
                         "busy_ms": round(upd["busy_ms"], 3),
                         "mean_launch_us": round(mean_s * 1e6, 2)},
            "kernel_ms": {k: round(v["total_ms"], 3) for k, v in prof_p.items()},
        }
        log(f"{PREC_NAMES[prec]}: " + json.dumps(mfma[PREC_NAMES[prec]]))
        del plan_p
    for td in tds:
        td.desc.precision = 0

    single = None
    if not args.no_single:
        single = single_tile_bench(fpm)
        log("single tile: " + json.dumps(single))

    paper = None
    if not args.no_single:
        paper = paper_workload_bench(fpm)
        log("paper workload: " + json.dumps(paper))

    online = None
    if not args.no_online:
        online = online_bench(fpm, tds, I, args.tiles_per_side)
        log("online: " + json.dumps(online))

    uneven = None
    if args.uneven_tiles > 0:
        uneven = uneven_bench(fpm, args.uneven_tiles, steps=1, warmup=1)
        log("uneven batch: " + json.dumps(uneven))

    serving = None
    if not args.no_serving:
        serving = serving_bench(fpm)
        log("serving: " + json.dumps(serving))
    cpu, accuracy = (None, None) if args.no_cpu_baseline else cpu_baseline(fpm)
    if accuracy is not None:
        log("accuracy vs FP64 oracle: " + json.dumps(accuracy))
    info = plan.infos[0]
    out = {
        "metric": "LED-tile updates/sec (FP32 vs MFMA DFT) + p50/p99 request latency",
        "value": round(value, 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"full-field {args.tiles_per_side}x{args.tiles_per_side} tiles of "
                        f"{info.n} px, 15x15 LEDs, {info.N}x{info.N} spectrum per tile, "
                        f"{args.iterations} iterations, LED groups, pupil recovery, FP32 FFT",
            "tiles": plan.ntiles, "n": info.n, "N": info.N, "leds": info.L,
            "iterations": args.iterations, "updates_per_step": updates,
            "schedule": "led_groups", "precision": "fp32_fft",
            "graph": not args.no_graph,
            # the library's default for a plan of one FP32 class up to 128 px
            "chains": int(os.environ.get("FPM_CHAINS", str(min(4, plan.ntiles)))),
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "rel_l2_vs_oracle": accuracy,
        "mfma": mfma,
        "stitch": stitch,
        "single_tile": single,
        "online": online,
        "paper_workload": paper,
        "host_mode": host_mode,
        "uneven_batch": uneven,
        "serving": serving,
        "kernel_ms": {k: round(v["total_ms"], 3) for k, v in prof.items()},
        "kernel_busy_ms": {k: round(v["busy_ms"], 3) for k, v in prof.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
