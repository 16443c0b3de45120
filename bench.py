"""Throughput of the RGB-D GMM + PBAS classify-and-update step on one MI355X.

A step pushes one 1280x720 RGB-D frame through each of 8 GMM models (Kc = Kd = 5) and
4 PBAS models (N = 35): one launch per kind, state read and written once each, masks
written.  Frames are synthetic (8 moving objects with shadows), distinct, generated
before the timed region and resident in HBM; every model first runs untimed through the
sequence's first frames (default 100) so that the timed frames meet it in its steady
state.  Then the 32-stream serving workload gives p50 / p99 frame latency, and the CPU
oracle is timed on a bounded sample.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
H, W = 720, 1280
KC = KD = 5
N_PBAS = 35


def gmm_bytes_per_px(Kc=KC, Kd=KD):
    # state read + written once (20 B per colour Gaussian, 12 B per depth Gaussian)
    # + 3 B RGB + 2 B depth in + 1 B mask out
    return 2 * (20 * Kc + 12 * Kd) + 6


def pbas_bytes_per_px(N=N_PBAS):
    # N sample words read; R, T (16 B each) and S (8 B) read + written; input and mask.
    # The sparse sample / D-history slot writes are not counted.
    return 4 * N + 2 * (16 + 16 + 8) + 6


def pbas_static_floor_bytes_per_px(N=N_PBAS, T=2.0, channels=4, gran=64, write_gran=None, H=H, W=W):
    """Expected HBM bytes per pixel-frame that the PBAS step must move at `gran`-byte
    sectors on a static background, where every pixel is background and T sits at its
    lower bound, so each channel self-updates and fires into a neighbour with
    probability u = 1/T, each at a uniform slot among N (the per-channel draws of the
    method).  State layout of the step kernel: sample quads of 16 B per pixel (4 pixels
    per 64-byte sector), D history one 4-byte word per slot and pixel (16 pixels per
    sector).  Counted: every sample quad, T, S, input and the fire bytes with their tile
    halo read (R stays at its lower bound, which the fire bytes flag, so it is not read);
    the D-history sectors holding a self-update's old byte read; the
    sample-quad sectors a self-update or an incoming neighbour write lands in written,
    with the quad holding the previous-value slot (N >= 33 not a multiple of 4, else a
    plane of its own); mask and fire bytes written.  Left out, as data-dependent: D, S,
    R and T writes (on a static background R and T do not move; D and S move only where
    d_min differs from the byte it replaces).  Reads are counted in `gran`-byte sectors,
    writes in `write_gran`-byte ones (default: the same)."""
    wg = write_gran or gran
    u = 1.0 / T
    pad = N >= 33 and N % 4 != 0
    nq = (N + 3) // 4
    dpx, qpx = gran // 4, wg // 16
    # a pixel reads D slot k if one of its channels self-updates into slot k
    p_px = 1.0 - (1.0 - u / N) ** channels
    d_read = 4.0 * N * (1.0 - (1.0 - p_px) ** dpx)
    # writes landing in a sector of qpx pixels: self (qpx*C Bernoulli(u)) and incoming
    # (each of the 8 neighbours of each pixel-channel fires toward it with u/8)
    s_write = 0.0
    for q in range(nq):
        slots = min(4, N - 4 * q)
        if pad and 4 * q <= N < 4 * q + 4:
            s_write += 16.0
            continue
        z = 1.0 - slots / N
        clean = (1.0 - u + u * z) ** (qpx * channels) * (1.0 - u / 8 + u / 8 * z) ** (8 * qpx * channels)
        s_write += 16.0 * (1.0 - clean)
    tiles_halo = ((64 + 2) * (4 + 2)) / (64 * 4)
    # R sits on its lower bound: flagged in the fire bytes, not read; T and S read
    reads = 16.0 * nq + (0 if pad else 4) + 24.0 + 5.0 + tiles_halo + d_read
    writes = s_write + (0 if pad else 4) + 2.0
    return {"total": reads + writes, "D_read": d_read, "samples_write": s_write + (0 if pad else 4),
            "reads": reads, "writes": writes}


PBAS_FLOOR_FILE = "pbas_traffic_floor_1280x720_n35.txt"


def pbas_floor_entry():
    """The PBAS traffic floor: counted from the oracle's run of the benchmark sequence
    (profiles/pbas_traffic_floor_1280x720_n35.txt, reads in 128-byte lines and writes in
    64-byte sectors, as the device requests them), and the closed form for a static
    background with T at its lower bound at the same granularities."""
    out = {}
    path = os.path.join(ROOT, "profiles", PBAS_FLOOR_FILE)
    if os.path.exists(path):
        kv = _kv(path)
        if "floor_bytes_per_px" in kv:
            out["floor_bytes_per_px"] = float(kv["floor_bytes_per_px"])
            out["floor_source"] = "profiles/" + PBAS_FLOOR_FILE
    st = pbas_static_floor_bytes_per_px(gran=128, write_gran=64)
    out["floor_static_T_lower_bytes_per_px"] = round(st["total"], 1)
    return out


def kernel_entry(avg_ms, bytes_per_px, gbs, profile, launches_per_step, models_per_launch, step_s):
    """Per-kernel figures of the default benchmark (None if the kernel did not run)."""
    if not launches_per_step:
        return None
    traffic = measured_traffic(profile)
    out = {"avg_ms": round(avg_ms, 5), "launches_per_step": launches_per_step,
           "models_per_launch": models_per_launch, "bytes_per_px": bytes_per_px,
           "GBs": round(gbs, 1), "traffic": traffic,
           "Mpx_per_s": round(models_per_launch * H * W / (avg_ms * 1e-3) / 1e6, 1),
           "frac": round(gbs / HBM_PEAK_GBS, 4),
           "share_of_step": round(launches_per_step * avg_ms * 1e-3 / step_s, 4)}
    if traffic is not None:
        out["GBs_from_traffic"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
        out["traffic_bytes_per_px"] = round(traffic / (models_per_launch * H * W), 1)
    if profile == PROFILE_FILES["pbas"]:
        out.update(pbas_floor_entry())
    return out


PROFILE_FILES = {"gmm": "gmm_step_1280x720_k5.txt", "pbas": "pbas_step_1280x720_n35.txt"}


def roofline_entry(kind, avg_ms, achieved_gbs, models_per_launch, bytes_per_px):
    """The roofline object of the dominant kernel.  achieved / frac count algorithmic bytes
    (the method's state read and written once, input and mask) per launch over the launch's
    average duration; traffic is the HBM bytes per launch rocprofv3 measured (read requests
    of 32, 64 and 128 bytes, and WRITE_SIZE), and *_from_traffic put those bytes over the
    same duration."""
    npx = H * W
    traffic = measured_traffic(PROFILE_FILES[kind])
    out = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kind + "_step",
           "algorithmic_bytes_per_launch": int(models_per_launch * bytes_per_px * npx),
           "algorithmic_bytes_per_px": bytes_per_px}
    if traffic is not None:
        tg = traffic / (avg_ms * 1e-3) / 1e9
        out.update(traffic_bytes_per_px=round(traffic / (models_per_launch * npx), 1),
                   achieved_from_traffic=round(tg, 1), frac_from_traffic=round(tg / HBM_PEAK_GBS, 4))
    if kind == "pbas":
        out.update(pbas_floor_entry())
    out["note"] = ("achieved and frac: algorithmic bytes per launch / average launch time (HIP events on the "
                   "launch stream); traffic: measured HBM bytes per launch (rocprofv3: read requests by size "
                   "plus WRITE_SIZE, profiles/" + PROFILE_FILES[kind] + "), achieved_from_traffic and "
                   "frac_from_traffic: those bytes over the same time")
    if traffic is not None and traffic < out["algorithmic_bytes_per_launch"]:
        out["note"] += ("; the algorithmic count has every state byte written once, while the kernel leaves "
                        "64-byte sectors that no pixel changed unwritten, so HBM moves fewer bytes than "
                        "that count and the algorithmic rate can reach or pass the peak: frac_from_traffic "
                        "is the rate HBM delivered")
    return out


def _kv(path):
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def measured_traffic(kernel_file: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the kernel source as it is now (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    kv = _kv(path)
    h = hashlib.sha256()
    for src in kv.get("sources", "").split():
        full = os.path.join(ROOT, src)
        if not os.path.isfile(full):
            return None
        h.update(open(full, "rb").read())
    if h.hexdigest()[:16] != kv.get("sources_sha256_16"):
        return None
    return float(kv["hbm_bytes_per_dispatch"])


def measured_traffic_per_model(kernel_file: str):
    """HBM bytes per model-frame: a profiled launch's bytes over the models it stepped."""
    t = measured_traffic(kernel_file)
    if t is None:
        return None
    return t / float(_kv(os.path.join(ROOT, "profiles", kernel_file)).get("models_per_dispatch", 1))


def _gen(args):
    from synth import Scene, preset
    t0, n = args
    sc = Scene(preset("hd_1280x720"))
    out = [sc.frame(t)[:2] for t in range(t0, t0 + n)]
    return np.stack([o[0] for o in out]), np.stack([o[1] for o in out])


def make_frames(n_frames: int, workers: int):
    from concurrent.futures import ProcessPoolExecutor
    chunks = [(i, min(8, n_frames - i)) for i in range(0, n_frames, 8)]
    if workers > 1:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            parts = list(ex.map(_gen, chunks))
    else:
        parts = [_gen(c) for c in chunks]
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def _oracle_stream(rgb, depth, n_g, n_p, barrier=None):
    """One independent stream of the oracle: PBAS fill frames untimed, then n_g GMM and
    n_p PBAS updating frames timed.  Returns (GMM s/frame, PBAS s/frame)."""
    from oracle.gmm import GmmParams, GmmRef
    from oracle.pbas import PbasParams, PbasRef
    g = GmmRef(H, W, GmmParams(Kc=KC, Kd=KD))
    p = PbasRef(H, W, PbasParams(N=N_PBAS))
    for k in range(N_PBAS):
        p.step(rgb[k % len(rgb)], depth[k % len(depth)])
    g.step(rgb[0], depth[0])
    if barrier is not None:
        barrier.wait()
    t0 = time.perf_counter()
    for i in range(n_g):
        g.step(rgb[(i + 1) % len(rgb)], depth[(i + 1) % len(depth)])
    tg = time.perf_counter() - t0
    t0 = time.perf_counter()
    for i in range(n_p):
        p.step(rgb[i % len(rgb)], depth[i % len(depth)])
    tp = time.perf_counter() - t0
    return tg / n_g, tp / n_p


def _oracle_small_configs():
    """The oracle on one thread at the two parity workloads: GMM Kc = Kd = 3 at 320x240 and
    PBAS N = 20 at 640x480 (its 20 fill frames untimed)."""
    from oracle.gmm import GmmParams, GmmRef
    from oracle.pbas import PbasParams, PbasRef
    from synth import Scene, preset
    res = []
    sc = Scene(preset("gmm_320x240"))
    fr = [sc.frame(t)[:2] for t in range(21)]
    g = GmmRef(240, 320, GmmParams(Kc=3, Kd=3))
    g.step(*fr[0])
    t0 = time.perf_counter()
    for f in fr[1:]:
        g.step(*f)
    dt = (time.perf_counter() - t0) / 20
    res.append({"workload": "GMM Kc=Kd=3, 320x240", "frames": 20, "value": round(240 * 320 / dt / 1e6, 4),
                "unit": "Mpixel-frames/s", "cores": 1})
    sc = Scene(preset("pbas_640x480"))
    fr = [sc.frame(t)[:2] for t in range(28)]
    p = PbasRef(480, 640, PbasParams(N=20))
    for f in fr[:20]:
        p.step(*f)
    t0 = time.perf_counter()
    for f in fr[20:]:
        p.step(*f)
    dt = (time.perf_counter() - t0) / 8
    res.append({"workload": "PBAS N=20, 640x480", "frames": 8, "value": round(480 * 640 / dt / 1e6, 4),
                "unit": "Mpixel-frames/s", "cores": 1})
    return res


_PAR = {}


def _oracle_stream_worker(i):
    return _oracle_stream(_PAR["rgb"], _PAR["depth"], _PAR["n_g"], _PAR["n_p"], _PAR["barrier"])


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rgb, depth, procs: int):
    """The oracle, untuned, on a bounded sample of the same workload (host cores): one
    stream on one thread, then `procs` independent streams in as many forked processes
    started together (their summed rates)."""
    n_g, n_p = 12, 8
    sg, sp = _oracle_stream(rgb, depth, n_g, n_p)
    step_s = sg + sp
    out = dict(value=round(2 * H * W / step_s / 1e6, 4), unit="Mpixel-frames/s", cores=1,
               kind="oracle",
               sample=f"numpy oracle, 1280x720: {n_g} GMM K=5 frames ({sg * n_g:.1f} s) + {n_p} PBAS "
                      f"N=35 updating frames ({sp * n_p:.1f} s), one host thread; step = one GMM + "
                      f"one PBAS frame; CPU: {cpu_model()}")
    out["configs"] = _oracle_small_configs()
    if procs > 1:
        import multiprocessing as mp
        ctx = mp.get_context("fork")  # the workers only run numpy
        pn_g, pn_p = 3, 2
        _PAR.update(rgb=rgb[:8], depth=depth[:8], n_g=pn_g, n_p=pn_p, barrier=ctx.Barrier(procs))
        t0 = time.perf_counter()
        with ctx.Pool(procs) as pool:
            res = pool.map(_oracle_stream_worker, range(procs))
        wall = time.perf_counter() - t0
        _PAR.clear()
        agg = sum(2 * H * W / (a + b) for a, b in res) / 1e6
        out["parallel"] = dict(value=round(agg, 4), unit="Mpixel-frames/s", cores=procs,
                               sample=f"{procs} independent oracle streams in {procs} processes started "
                                      f"together, each {pn_g} GMM + {pn_p} PBAS frames of 1280x720; "
                                      f"summed per-stream rates ({wall:.1f} s wall)")
    return out


SERVE_SIZES = [(240, 424)] * 12 + [(480, 640)] * 12 + [(720, 1280)] * 8


def serving_run(warm_s: float, seconds: float, saturate_s: float = 0.0) -> dict:
    """The 32-stream serving workload: 12x 424x240, 12x 640x480, 8x 1280x720, even streams
    GMM K=5, odd PBAS N=20, frames at 30 fps (random phase, +-5 ms jitter), after `warm_s`
    seconds of the same load untimed (PBAS fills its samples); with saturate_s > 0 the same
    streams then run at saturation (every ring kept full) for the aggregate capacity."""
    import threading
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server, StreamLoad, run_camera_load
    from synth import Scene, preset
    srv = Server(64 << 30, 32)
    loads = []
    for i, (h, w) in enumerate(SERVE_SIZES):
        if i % 2 == 0:
            p = fgs.fgs_gmm_params_default()
            p.Kc = p.Kd = 5
            algo = fgs.FGS_GMM
        else:
            p = fgs.fgs_pbas_params_default()
            p.N = 20
            p.seed = 7000 + i
            algo = fgs.FGS_PBAS
        sid = srv.open(algo, h, w, p)
        sc = Scene(preset("hd_1280x720", H=h, W=w, seed=300 + i))
        loads.append(StreamLoad(sid, [sc.frame(t)[:2] for t in range(4)]))
    run_camera_load(srv, [StreamLoad(l.sid, l.frames) for l in loads], duration_s=warm_s, seed=1)
    srv.reset_stats()
    lat, wall = run_camera_load(srv, loads, duration_s=seconds, seed=2)
    st = srv.stats()
    offered = sum(h * w for h, w in SERVE_SIZES) * 30 / 1e6
    out = {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
           "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
           "max_ms": round(float(lat.max()) * 1e3, 4),
           "frames": int(lat.size), "frame_period_ms": round(1000 / 30, 3),
           "served_Mpx_frames_per_s": round(st["mpix_frames_per_s"], 2),
           "offered_Mpx_frames_per_s": round(offered, 2),
           "frames_per_batch": round(st["mean_batch_frames"], 3),
           "seconds": seconds, "warmup_seconds": warm_s,
           "workload": "32 streams: 12x 424x240, 12x 640x480, 8x 1280x720; even GMM K=5, odd PBAS N=20; "
                       "30 fps, +-5 ms jitter; latency = frame arrival to mask on the host"}
    if saturate_s > 0:
        # saturation: one thread per stream keeps its ring full for the same duration
        srv.reset_stats()
        stop = [False]

        def pump(ld):
            tickets, k = [], 0
            while not stop[0]:
                rgb, dep = ld.frames[k % len(ld.frames)]
                try:
                    tickets.append(srv.submit(ld.sid, rgb, dep))
                    k += 1
                except fgs.FgsError:
                    srv.wait(tickets.pop(0))
            for t in tickets:
                srv.wait(t)
        ths = [threading.Thread(target=pump, args=(ld,)) for ld in loads]
        for t in ths:
            t.start()
        time.sleep(saturate_s)
        stop[0] = True
        for t in ths:
            t.join()
        sat = srv.stats()
        out["saturated"] = {"Mpx_frames_per_s": round(sat["mpix_frames_per_s"], 1),
                            "frames_per_batch": round(sat["mean_batch_frames"], 2),
                            "p50_ms": round(sat["p50_latency_s"] * 1e3, 3),
                            "p99_ms": round(sat["p99_latency_s"] * 1e3, 3)}
    srv.destroy()
    return out


def serving_main(args):
    """--serving: the serving workload alone, p99 latency as the value."""
    r = serving_run(1.0, args.serve_seconds, saturate_s=args.serve_seconds)
    out = {
        "metric": "p99 frame latency (32 mixed-resolution RGB-D streams at 30 fps)",
        "value": r["p99_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "higher_is_better": False,
        "frames": r["frames"],
        "p50_ms": r["p50_ms"],
        "max_ms": r["max_ms"],
        "frame_period_ms": r["frame_period_ms"],
        "served_Mpx_frames_per_s": r["served_Mpx_frames_per_s"],
        "offered_Mpx_frames_per_s": r["offered_Mpx_frames_per_s"],
        "frames_per_batch": r["frames_per_batch"],
        "saturated": r["saturated"],
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": r["workload"], "seconds": args.serve_seconds},
    }
    print(json.dumps(out), flush=True)


def adjoint_main(args):
    """GMM adjoint on the 640x480, K=3, 64-frame window (checkpoint every 16 frames): time of
    one forward + backward (one Adam step of theta = (alpha, lambda, w_d))."""
    import torch
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.adjoint import GmmWindow, GmmWindowFunction, window_bce_loss
    from synth import Scene, preset
    T, Hh, Ww = 64, 480, 640
    rgb, dep, gt = Scene(preset("adjoint_640x480")).frames(0, T)
    r = torch.from_numpy(rgb).cuda()
    d = torch.from_numpy(dep.view(np.int16)).cuda()
    g = torch.from_numpy(gt).cuda()
    p = fgs.fgs_gmm_params_default()
    win = GmmWindow(T, Hh, Ww, p, checkpoint_every=16)
    theta = torch.tensor([0.01, 2.5, 1.0], device="cuda", requires_grad=True)
    opt = torch.optim.Adam([theta], lr=1e-3)

    def step():
        opt.zero_grad()
        Z, has = GmmWindowFunction.apply(theta, r, d, win)
        loss = window_bce_loss(Z, has, g)
        loss.backward()
        opt.step()
        with torch.no_grad():   # keep theta in its valid range
            theta.clamp_(min=torch.tensor([1e-4, 0.5, 0.0], device="cuda"),
                         max=torch.tensor([0.5, 10.0, 10.0], device="cuda"))
        return loss
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    steps = max(5, args.steps // 10)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    tf = tb = 0.0
    for _ in range(steps):
        e[0].record()
        Z, has = win.forward(theta.detach(), r, d)
        e[1].record()
        win.backward(theta.detach(), r, d, torch.zeros_like(Z))
        e[2].record()
        torch.cuda.synchronize()
        tf += e[0].elapsed_time(e[1])
        tb += e[1].elapsed_time(e[2])
    t0 = time.perf_counter()
    for _ in range(steps):
        loss = step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    px = T * Hh * Ww
    out = {"metric": "GMM adjoint window step (forward + backward + Adam)", "value": round(wall * 1e3, 3),
           "unit": "ms", "higher_is_better": False, "n_gpus": 1, "steps": steps,
           "forward_ms": round(tf / steps, 3), "backward_ms": round(tb / steps, 3),
           "forward_Mpx_frames_per_s": round(px / (tf / steps * 1e-3) / 1e6, 1),
           "backward_Mpx_frames_per_s": round(px / (tb / steps * 1e-3) / 1e6, 1),
           "loss": round(float(loss), 5), "theta": [round(float(x), 6) for x in theta.detach().cpu()],
           "dtype": "f32 (fp64 gradient reduction)", "data": "synthetic",
           "config": {"workload": "640x480, K=3, 64-frame window, checkpoint every 16 frames, BCE on sigmoid(Z)"}}
    win.close()
    print(json.dumps(out), flush=True)


MEDIAN_R = 4   # the base PBAS method's 9x9 median window


def eval_main(args):
    """Evaluation counters on 1280x720: per-frame confusion counts of a GMM K=5 model's
    mask against ground truth accumulated on the device, the Sec. 5 indicators from them,
    and the counting kernel timed on its own (2 B/px: mask + ground truth).  Beside them,
    the median post-filter: the indicators of the 9x9-filtered masks and the filter kernel
    timed on its own at radii 1, 4 and 7 (2 B/px: mask in, mask out)."""
    import torch
    from paper_2002_00250_amd import fgs
    from synth import Scene, preset
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    sc = Scene(preset("hd_1280x720"))
    frames = [sc.frame(t) for t in range(32)]
    rgb = torch.from_numpy(np.stack([f[0] for f in frames])).to(dev)
    dep = torch.from_numpy(np.stack([f[1] for f in frames]).view(np.int16)).to(dev)
    gt = torch.from_numpy(np.stack([f[2] for f in frames])).to(dev)
    gp = fgs.fgs_gmm_params_default()
    gp.Kc, gp.Kd = KC, KD
    m = fgs.Model(fgs.FGS_GMM, H, W, gp, stream=stream)
    med = torch.empty((H, W), dtype=torch.uint8, device=dev)
    med_counts = np.zeros(4, np.int64)
    for t in range(len(frames)):
        fgs.fgs_push_frame(m.handle, rgb[t].data_ptr(), 3 * W, dep[t].data_ptr(), 2 * W, fgs.FGS_MEM_DEVICE)
        if t >= 8:
            m.eval_accumulate(gt[t])
            fgs.fgs_mask_median(m.mask_ptr, W, med.data_ptr(), W, H, W, MEDIAN_R, stream.cuda_stream)
            fm, g = med.cpu().numpy() != 0, gt[t].cpu().numpy() != 0
            med_counts += [np.sum(fm & g), np.sum(~fm & ~g), np.sum(fm & ~g), np.sum(~fm & g)]
    counts = m.eval_read(reset=True)
    med_us = {}
    for r in (1, MEDIAN_R, 7):
        for _ in range(20):
            fgs.fgs_mask_median(m.mask_ptr, W, med.data_ptr(), W, H, W, r, stream.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fgs.fgs_mask_median(m.mask_ptr, W, med.data_ptr(), W, H, W, r, stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        med_us[r] = e0.elapsed_time(e1) / args.steps * 1e3
    K = args.steps
    g_last = gt[-1].data_ptr()        # one stream throughout: the raw call, no stream waits
    for _ in range(20):
        fgs.fgs_eval_accumulate(m.handle, g_last, W, fgs.FGS_MEM_DEVICE)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(K):
        fgs.fgs_eval_accumulate(m.handle, g_last, W, fgs.FGS_MEM_DEVICE)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / K * 1e3
    m.close()
    ind = indicators_from(counts)
    out = {"metric": "evaluation counters: confusion-count kernel time per 1280x720 frame", "value": round(us, 3),
           "unit": "us", "higher_is_better": False, "n_gpus": 1, "steps": K,
           "GBs": round(2 * H * W / (us * 1e-6) / 1e9, 1),
           "counts_tp_tn_fp_fn": list(counts), "indicators": {k: round(v, 5) for k, v in ind.items()},
           "median_filter": {"us_per_frame": {f"r{r}": round(v, 3) for r, v in med_us.items()},
                             "GBs": {f"r{r}": round(2 * H * W / (v * 1e-6) / 1e9, 1) for r, v in med_us.items()},
                             f"indicators_r{MEDIAN_R}": {k: round(v, 5) for k, v in
                                                         indicators_from([int(x) for x in med_counts]).items()}},
           "dtype": "u8", "data": "synthetic",
           "config": {"workload": "GMM Kc=Kd=5 1280x720, frames 8..31 scored against ground truth"}}
    print(json.dumps(out), flush=True)


def indicators_from(c):
    tp, tn, fp, fn = c
    d = lambda a, b: a / b if b else float("nan")
    return {"PWC": 100.0 * d(fn + fp, tp + tn + fp + fn), "FNR": d(fn, tp + fn), "FPR": d(fp, fp + tn),
            "Si": d(tp, tp + fp + fn)}


def table1_main(args):
    """The resolutions of the paper's performance table (RGB / depth: 480p/480p, 720p/480p,
    720p/720p, 1080p/720p; depth upscaled in the kernel when smaller), one stream at a time,
    with the paper's GMM settings (7 colour + 3 depth Gaussians, learning rate 0.001) and PBAS
    N = 20.  Frames per second of each kernel, device-resident input."""
    import torch
    from paper_2002_00250_amd import fgs
    from synth import Scene, preset
    cols = [("480p/480p", (480, 640), (480, 640)), ("720p/480p", (720, 1280), (480, 640)),
            ("720p/720p", (720, 1280), (720, 1280)), ("1080p/720p", (1080, 1920), (720, 1280))]
    paper_fps = {"Jetson TX2": [28, 11, 9, 6], "GTX 1050m": [30, 18, 16, 10], "RTX 2070 (camera-capped)": [30, 30, 30, 30]}
    st = torch.cuda.Stream()
    torch.cuda.set_stream(st)
    res = {}
    for name, (H, W), (Hd, Wd) in cols:
        sc = Scene(preset("hd_1280x720", H=H, W=W))
        fr = [sc.frame(t)[:2] for t in range(8)]
        ys, xs = (np.arange(Hd) * H) // Hd, (np.arange(Wd) * W) // Wd
        rgb = torch.from_numpy(np.stack([f[0] for f in fr])).cuda()
        dep = torch.from_numpy(np.ascontiguousarray(np.stack([f[1][ys][:, xs] for f in fr])).view(np.int16)).cuda()
        gp = fgs.fgs_gmm_params_default()
        gp.Kc, gp.Kd, gp.alpha = 7, 3, 0.001
        pp = fgs.fgs_pbas_params_default()
        pp.N = 20
        row = {}
        for algo, prm, tag in ((fgs.FGS_GMM, gp, "gmm_7_3"), (fgs.FGS_PBAS, pp, "pbas_20")):
            m = fgs.Model(algo, H, W, prm, stream=st)

            def push(i):
                fgs.fgs_push_frame_scaled(m.handle, rgb[i % 8].data_ptr(), 3 * W, dep[i % 8].data_ptr(), 2 * Wd,
                                          Hd, Wd, fgs.FGS_MEM_DEVICE)
            for i in range(40):
                push(i)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            n = 200
            e0.record(st)
            for i in range(n):
                push(40 + i)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / n
            row[tag] = {"fps": round(1000.0 / ms, 1), "us_per_frame": round(ms * 1e3, 2),
                        "Mpx_frames_per_s": round(H * W / (ms * 1e-3) / 1e6, 1)}
            m.close()
        res[name] = row
    out = {"metric": "frames per second per stream at the paper's Table 1 resolutions", "unit": "fps",
           "higher_is_better": True, "n_gpus": 1, "columns": res,
           "paper_fps_context_only": paper_fps, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "one stream; GMM Kc=7 Kd=3 alpha=0.001 and PBAS N=20; depth upscaled in-kernel "
                                  "when its resolution is lower; 480p = 640x480"}}
    print(json.dumps(out), flush=True)


PROFILE_CMD = ("cd /tmp && TMPDIR=/tmp rocprofv3 {opts} --output-format csv -d $OUT/{sub} -o {name} -- "
               "python3 $REPO/bench.py --steps 200 --no-cpu-baseline --no-serving")
PROFILE_PASSES = {  # sub-directory: rocprofv3 options (each --pmc pass in a run of its own)
    "stats": "--kernel-trace --stats",
    "pmc_FETCH_SIZE": "--pmc FETCH_SIZE",
    "pmc_WRITE_SIZE": "--pmc WRITE_SIZE",
    "pmc_rdreq": "--pmc TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum",
    "pmc_wrreq": "--pmc TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum",
    "pmc_sq": "--pmc SQ_ACTIVE_INST_VALU SQ_INSTS_VALU SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_WAIT_INST_ANY "
              "SQ_ACTIVE_INST_VMEM GRBM_GUI_ACTIVE",
}
SQ_COUNTERS = ["GRBM_GUI_ACTIVE", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_VMEM", "SQ_BUSY_CYCLES", "SQ_INSTS_VALU",
               "SQ_WAIT_INST_ANY", "SQ_WAVES", "SQ_WAVE_CYCLES"]
STEP_KERNELS = {  # summary file: (kernel name in the trace, models per dispatch, sources, alg. B/px)
    "gmm_step_1280x720_k5.txt": ("gmm_step_kernel<8, 5, 5, true, false, 1>", 8,
                                 ["paper_2002_00250_amd/csrc/gmm_kernels.hip", "paper_2002_00250_amd/csrc/gmm_device.h",
                                  "paper_2002_00250_amd/csrc/device_common.h",
                                  "paper_2002_00250_amd/csrc/fgs_internal.h"], gmm_bytes_per_px()),
    "pbas_step_1280x720_n35.txt": ("pbas_step_kernel<8, 36, true>", 4,
                                   ["paper_2002_00250_amd/csrc/pbas_kernels.hip",
                                    "paper_2002_00250_amd/csrc/pbas_device.h",
                                    "paper_2002_00250_amd/csrc/device_common.h",
                                    "paper_2002_00250_amd/csrc/fgs_internal.h"], pbas_bytes_per_px()),
}
COPY_KERNEL = "copy_kernel"
PROFILE_STEPS = 200    # the --steps of the profile command: each step kernel's last dispatches
COPY_BYTES = 1 << 30   # the probe's bytes read (and written) per dispatch


def _csv_rows(directory: str, suffix: str):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return rows


def _counter_means(directory: str, last: int | None = None):
    """{kernel name: {counter: mean value per dispatch}} from a --pmc pass; with `last`,
    over each kernel's last `last` dispatches only (those of the timed steps)."""
    acc = {}
    for r in _csv_rows(directory, "counter_collection.csv"):
        k = r["Kernel_Name"]
        c = r["Counter_Name"]
        d = acc.setdefault(k, {}).setdefault(c, {})
        i = int(r["Dispatch_Id"])
        d[i] = d.get(i, 0.0) + float(r["Counter_Value"])
    out = {}
    for k, cs in acc.items():
        out[k] = {}
        for c, v in cs.items():
            vals = [v[i] for i in sorted(v)][-last:] if last else list(v.values())
            out[k][c] = sum(vals) / len(vals)
    return out


def _trace_durations(directory: str, last: int | None = None):
    """{kernel name: (mean duration in ns, dispatches)} from a kernel trace; with `last`, over
    each kernel's last `last` dispatches."""
    per = {}
    for r in _csv_rows(directory, "kernel_trace.csv"):
        per.setdefault(r["Kernel_Name"], []).append(
            (int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = {}
    for k, v in per.items():
        v = [d for _, d in sorted(v)]
        v = v[-last:] if last else v
        out[k] = (sum(v) / len(v), len(v))
    return out


def _short_kernel_name(name: str) -> str:
    """'void ns::(anonymous namespace)::k<1, 2>(args)' -> 'k<1, 2>'."""
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]
    n = n.replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            n = n[:i]
            break
    head = n if "<" not in n else n[:n.find("<")]
    return n[head.rfind("::") + 2:] if "::" in head else n


def _find_kernel(table: dict, name: str):
    for k in table:
        if _short_kernel_name(k) == name:
            return table[k]
    raise KeyError(f"kernel {name} not in the profile ({sorted(table)[:6]} ...)")


def summarize_profiles(directory: str) -> None:
    """Write profiles/*_1280x720_*.txt and the kernel statistics table from the rocprofv3 CSV
    output of PROFILE_PASSES (each under directory/<sub>).  HBM bytes: FETCH_SIZE and
    WRITE_SIZE, each divided by what the counter reads for the plain copy kernel of the same
    runs (FETCH_SIZE counts a 128-byte read request as 64 bytes on this device); the read
    requests by size (32, 64 and 128 B) cross-check the reads."""
    import hashlib
    stats = {r["Name"]: r for r in _csv_rows(os.path.join(directory, "stats"), "kernel_stats.csv")}
    timed = _trace_durations(os.path.join(directory, "stats"), PROFILE_STEPS)
    pmc = {sub: _counter_means(os.path.join(directory, sub), PROFILE_STEPS) for sub in PROFILE_PASSES
           if sub != "stats" and (sub != "pmc_sq" or os.path.isdir(os.path.join(directory, sub)))}
    cmds = [PROFILE_CMD.format(opts=o, sub=s, name="bench" if s == "stats" else "run")
            for s, o in PROFILE_PASSES.items()]
    cmd_text = "commands:\n" + "\n".join("  " + c for c in cmds) + \
        "\n  python3 $REPO/bench.py --summarize-profiles $OUT\n" \
        "($REPO = the repository root, $OUT = an output directory; each --pmc pass in its own run)\n"

    def req_bytes(kern):
        c = _find_kernel(pmc["pmc_rdreq"], kern)
        return (32 * c["TCC_EA0_RDREQ_32B_sum"] + 64 * c["TCC_EA0_RDREQ_64B_sum"]
                + 128 * c["TCC_EA0_RDREQ_128B_sum"])
    copy_fetch = _find_kernel(pmc["pmc_FETCH_SIZE"], COPY_KERNEL)["FETCH_SIZE"] * 1024  # its 13 dispatches
    copy_write = _find_kernel(pmc["pmc_WRITE_SIZE"], COPY_KERNEL)["WRITE_SIZE"] * 1024
    copy_req = req_bytes(COPY_KERNEL)
    for fname, (kern, models, sources, alg) in STEP_KERNELS.items():
        h = hashlib.sha256()
        for src in sources:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        st = _find_kernel(stats, kern)
        avg_ns, n_timed = _find_kernel(timed, kern)
        fetch = _find_kernel(pmc["pmc_FETCH_SIZE"], kern)["FETCH_SIZE"] * 1024
        write = _find_kernel(pmc["pmc_WRITE_SIZE"], kern)["WRITE_SIZE"] * 1024
        rq = _find_kernel(pmc["pmc_rdreq"], kern)
        wq = _find_kernel(pmc["pmc_wrreq"], kern)
        req_read = req_bytes(kern)
        # HBM bytes: each counter divided by what it reads for the copy of known size
        fetch_scale = copy_fetch / COPY_BYTES
        write_scale = copy_write / COPY_BYTES
        read = fetch / fetch_scale
        write = write / write_scale
        npx = models * H * W
        lines = [
            f"# {kern} on 1280x720 frames (benchmark workload: one dispatch steps {models} models)", "",
            f"kernel: {kern}",
            f"sources: {' '.join(sources)}",
            f"sources_sha256_16: {h.hexdigest()[:16]}",
            f"avg_duration_ns: {avg_ns:.0f}",
            f"timed_dispatches: {n_timed}",
            f"calls: {st['Calls']}",
            f"avg_duration_all_calls_ns: {float(st['AverageNs']):.0f}",
            f"models_per_dispatch: {models}",
            f"read_requests_per_dispatch: 32B {rq['TCC_EA0_RDREQ_32B_sum']:.0f}, 64B {rq['TCC_EA0_RDREQ_64B_sum']:.0f}, "
            f"128B {rq['TCC_EA0_RDREQ_128B_sum']:.0f}",
            f"write_requests_per_dispatch: all {wq['TCC_EA0_WRREQ_sum']:.0f}, 64B {wq['TCC_EA0_WRREQ_64B_sum']:.0f}",
            f"fetch_size_kib_per_dispatch: {fetch / 1024:.0f}",
            f"write_size_kib_per_dispatch: {_find_kernel(pmc['pmc_WRITE_SIZE'], kern)['WRITE_SIZE']:.0f}",
            f"fetch_scale: {fetch_scale:.4f}",
            f"write_scale: {write_scale:.4f}",
            f"read_bytes_per_dispatch: {read:.0f}",
            f"write_bytes_per_dispatch: {write:.0f}",
            f"read_bytes_from_request_sizes: {req_read:.0f}",
            f"hbm_bytes_per_dispatch: {read + write:.0f}",
            f"hbm_bytes_per_pixel: {(read + write) / npx:.1f}",
            f"read_bytes_per_pixel: {read / npx:.1f}",
            f"write_bytes_per_pixel: {write / npx:.1f}",
            f"algorithmic_bytes_per_pixel: {alg}",
            f"hbm_GBs_at_avg_duration: {(read + write) / avg_ns:.1f}",
            "",
            f"Durations and counters are averages over the kernel's last {PROFILE_STEPS} dispatches, those of the "
            f"timed steps (the first ones step the untimed start and warm-up frames); avg_duration_all_calls_ns "
            f"covers every dispatch.",
            "",
            f"HBM bytes = FETCH_SIZE / fetch_scale + WRITE_SIZE / write_scale, the scales being what the counters "
            f"read on the plain copy kernel of the same runs ({COPY_KERNEL}, {COPY_BYTES >> 20} MiB read and written "
            f"per dispatch): FETCH_SIZE {copy_fetch / COPY_BYTES:.4f} x the bytes read (it counts a 128-byte read "
            f"request as 64 bytes), WRITE_SIZE {copy_write / COPY_BYTES:.4f} x the bytes written.  Cross-check: the "
            f"read requests by size (32, 64, 128 B) give {req_read:.0f} read bytes per dispatch "
            f"({copy_req / COPY_BYTES:.4f} x the copy's bytes read).",
            "",
            cmd_text,
        ]
        with open(os.path.join(ROOT, "profiles", fname), "w") as fh:
            fh.write("\n".join(lines))
    if "pmc_sq" in pmc:
        sq = ["# SQ counters of the benchmark command's step kernels (1280x720, GMM K=5 + PBAS N=35)", "",
              "command: " + [c for c in cmds if "SQ_" in c][0],
              "($REPO = the repository root, $OUT = an output directory)", "",
              "Averages per dispatch.  GRBM_GUI_ACTIVE is summed over the 8 XCDs (it reads about 8x the",
              "dispatch's cycles), so the per-XCD busy cycles are GRBM_GUI_ACTIVE / 8.  A wave64 VALU",
              "instruction occupies its SIMD for 4 cycles.  Derived:",
              "  VALU busy = SQ_ACTIVE_INST_VALU * 4 / 1024 SIMDs / (GRBM_GUI_ACTIVE / 8)",
              "  waiting   = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES (share of wave time spent waiting on",
              "              outstanding memory and other dependencies; same units, unit-free)",
              "  VALU instructions per wavefront = SQ_INSTS_VALU / SQ_WAVES"]
        for fname, (kern, models, sources, alg) in STEP_KERNELS.items():
            h = hashlib.sha256()
            for src in sources:
                h.update(open(os.path.join(ROOT, src), "rb").read())
            c = _find_kernel(pmc["pmc_sq"], kern)
            busy = c["SQ_ACTIVE_INST_VALU"] * 4 / 1024 / (c["GRBM_GUI_ACTIVE"] / 8)
            sq += ["", f"kernel: {kern}", f"sources_sha256_16: {h.hexdigest()[:16]}"]
            sq += [f"  {k}: {c[k]:.0f}" for k in SQ_COUNTERS if k in c]
            sq += [f"  VALU busy: {100 * busy:.1f} %",
                   f"  waiting: {100 * c['SQ_WAIT_INST_ANY'] / c['SQ_WAVE_CYCLES']:.1f} %",
                   f"  VALU instructions per wavefront: {c['SQ_INSTS_VALU'] / c['SQ_WAVES']:.0f}"]
        with open(os.path.join(ROOT, "profiles", "sq_counters_1280x720_bench.txt"), "w") as fh:
            fh.write("\n".join(sq) + "\n")
    _write_stats_table(stats, "bench_1280x720_kernel_stats.md",
                       "rocprofv3 kernel statistics of the benchmark command (1280x720, GMM K=5 + PBAS N=35)",
                       cmds[0])
    short = os.path.join(directory, "stats_short")
    if os.path.isdir(short):
        _write_stats_table({r["Name"]: r for r in _csv_rows(short, "kernel_stats.csv")},
                           "bench_1280x720_short_run_kernel_stats.md",
                           "rocprofv3 kernel statistics of the default benchmark line at 20 steps (1280x720, "
                           "GMM K=5 + PBAS N=35, serving and the CPU baseline included)", SHORT_CMD)


SHORT_CMD = ("cd /tmp && TMPDIR=/tmp rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/stats_short "
             "-o bench -- python3 $REPO/bench.py --steps 20 --warmup 5")


def _write_stats_table(stats: dict, fname: str, title: str, cmd: str) -> None:
    tot = sum(float(r["TotalDurationNs"]) for r in stats.values())
    rows = sorted(stats.values(), key=lambda r: -float(r["TotalDurationNs"]))
    md = ["# " + title, "", "command: " + cmd, "($REPO = the repository root, $OUT = an output directory)", "",
          "| kernel | calls | avg ns | min ns | max ns | % time |", "|---|---|---|---|---|---|"]
    for r in rows:
        md.append(f"| {_short_kernel_name(r['Name'])} | {r['Calls']} | {float(r['AverageNs']):.0f} | {float(r['MinNs']):.0f} | "
                  f"{float(r['MaxNs']):.0f} | {100 * float(r['TotalDurationNs']) / tot:.2f} |")
    with open(os.path.join(ROOT, "profiles", fname), "w") as fh:
        fh.write("\n".join(md) + "\n")


MIX_MODES = [  # fgs_mix_probe modes: (mode, planes read, planes written back in place)
    (0, 10, 10), (1, 10, 5), (2, 10, 0), (3, 0, 10), (4, 9, 9)]


def mix_probe_main(args):
    """What HBM gives the step kernels' access shape without their arithmetic: float4 planes of
    8 x 1280x720 pixels (1.18 GB for 10 planes), one lane per pixel, non-temporal, read and
    written back in place in the mixes of MIX_MODES, beside the plain copy."""
    import torch
    from paper_2002_00250_amd import fgs
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(dev)
    npix = 8 * H * W
    buf = torch.zeros(10 * npix * 16, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    out = {"metric": "HBM GB/s of read/write mixes in the step kernels' access shape", "unit": "GB/s",
           "n_gpus": 1, "npix": npix, "modes": []}
    for mode, rp, wp in MIX_MODES:
        for _ in range(3):
            fgs.fgs_mix_probe(buf.data_ptr(), npix, mode, stream.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        reps = 20
        for _ in range(reps):
            fgs.fgs_mix_probe(buf.data_ptr(), npix, mode, stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        byts = (rp + wp) * 16 * npix
        out["modes"].append({"mode": mode, "planes_read": rp, "planes_written": wp, "bytes_per_px": (rp + wp) * 16,
                             "us": round(ms * 1e3, 1), "GBs": round(byts / (ms * 1e-3) / 1e9, 1)})
    del buf
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--start", type=int, default=300,
                    help="frames every model runs through untimed before the warm-up (PBAS fill frames "
                         "included), so that the timed frames come from a model in its steady state (PBAS's "
                         "R and T settle over the first ~300 frames of the sequence, and its step cost with "
                         "them)")
    ap.add_argument("--models", type=lambda v: tuple(int(x) for x in v.split(",")), default=(8, 4),
                    help="GMM,PBAS model counts stepped round-robin (default 8,4: 2.4 GB of live state)")
    ap.add_argument("--per-model", action="store_true",
                    help="one launch per model (fgs_push_frame) instead of one per kind (fgs_push_frames)")
    ap.add_argument("--streams", type=int, default=1,
                    help="streams the models are spread over (model j on stream j mod S); with S > 1 "
                         "kernels of different models overlap, and the roofline describes the whole step")
    ap.add_argument("--kind-streams", action="store_true",
                    help="one launch per kind and step as by default, the GMM launch and the PBAS launch "
                         "on two streams so that they overlap (the roofline describes the whole step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--cpu-procs", type=int, default=min(16, len(os.sched_getaffinity(0))),
                    help="processes for the aggregate oracle baseline (1: single thread only)")
    ap.add_argument("--serving", action="store_true", help="run the 32-stream serving workload instead")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--no-serving", action="store_true",
                    help="leave the serving workload (p50/p99 latency) out of the default line")
    ap.add_argument("--adjoint", action="store_true", help="time the GMM adjoint window step instead")
    ap.add_argument("--table1", action="store_true", help="time the paper's Table 1 resolutions instead")
    ap.add_argument("--eval", action="store_true", help="time the evaluation counters instead")
    ap.add_argument("--mix-probe", action="store_true",
                    help="time the read/write mixes of the step kernels' access shape (fgs_mix_probe) instead")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write the profiles/ summaries from the rocprofv3 output of the profile passes in DIR "
                         "(no GPU)")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(each camera stream is independent: sharding is by stream, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2002_00250_amd import fgs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    fgs.lib()
    if args.serving:
        serving_main(args)
        return
    if args.adjoint:
        adjoint_main(args)
        return
    if args.table1:
        table1_main(args)
        return
    if args.eval:
        eval_main(args)
        return
    if args.mix_probe:
        mix_probe_main(args)
        return

    # A dedicated stream (the legacy null stream has handle 0, which the library reads as
    # "create a private stream"); every launch and every timing event goes on it.
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    n_g, n_p = args.models
    L0 = n_g + n_p
    # every frame pushed is a distinct frame of the sequence: model j takes frame t + j at
    # step t, for t = 0 .. start + warmup + steps - 1
    F = args.start + args.warmup + args.steps + max(0, L0 - 1)
    rgb_h, dep_h = make_frames(F, args.workers)
    rgb = torch.from_numpy(rgb_h).to(dev)
    dep = torch.from_numpy(dep_h.view(np.int16)).to(dev)

    gp = fgs.fgs_gmm_params_default()
    gp.Kc, gp.Kd = KC, KD
    pp = fgs.fgs_pbas_params_default()
    pp.N = N_PBAS
    # Independent camera models stepped round-robin, their live state far beyond the
    # 256 MB Infinity Cache, so every launch runs against HBM.
    S = 2 if args.kind_streams else max(1, args.streams)
    streams = [stream] + [torch.cuda.Stream(dev) for _ in range(S - 1)]
    if args.kind_streams:   # every GMM model on the first stream, every PBAS model on the second
        g_st, p_st = [streams[0]] * n_g, [streams[1]] * n_p
    else:
        g_st, p_st = [streams[j % S] for j in range(n_g)], [streams[(n_g + j) % S] for j in range(n_p)]
    models = [(fgs.Model(fgs.FGS_GMM, H, W, gp, stream=g_st[j]), "gmm") for j in range(n_g)] + \
             [(fgs.Model(fgs.FGS_PBAS, H, W, pp, stream=p_st[j]), "pbas") for j in range(n_p)]
    live = sum(fgs.fgs_device_bytes(m.handle) for m, _ in models)
    rs, ds = 3 * W, 2 * W

    def push(j, i):   # model j sees the sequence from its own offset j
        f = i + j
        fgs.fgs_push_frame(models[j][0].handle, rgb[f].data_ptr(), rs, dep[f].data_ptr(), ds,
                           fgs.FGS_MEM_DEVICE)

    # A step pushes a frame to every GMM model, then to every PBAS model, on one stream:
    # by default one fgs_push_frames call per kind, i.e. one launch for up to 8 models
    # (--per-model: one launch each).  Two events per step (its start and the GMM -> PBAS
    # boundary) time each block; a kernel's average launch is its blocks' total over its
    # launches.  With the models on several streams the events on the first stream do not
    # bracket the others' work, so only the wall time of the steps is used.
    K = args.steps
    L = len(models)
    batched = (S == 1 or args.kind_streams) and not args.per_model
    g_launches = (-(-n_g // 8) if batched else n_g)
    p_launches = (-(-n_p // 8) if batched else n_p)

    def push_kind(js, i):
        if not batched:
            for j in js:
                push(j, i)
            return
        fs = [i + j for j in js]
        fgs.fgs_push_frames([models[j][0].handle for j in js], [rgb[f].data_ptr() for f in fs], [rs] * len(js),
                            [dep[f].data_ptr() for f in fs], [ds] * len(js))
    g_js, p_js = list(range(n_g)), list(range(n_g, L))
    # untimed: frames 0 .. start - 1 (the PBAS models' N fill frames among them), then the
    # warm-up steps
    for i in range(args.start + args.warmup):
        for js in (g_js, p_js):
            if js:
                push_kind(js, i)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * K + 1)]
    base = args.start + args.warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        ev[2 * s].record(stream)
        if g_js:
            push_kind(g_js, base + s)
        ev[2 * s + 1].record(stream)
        if p_js:
            push_kind(p_js, base + s)
    ev[2 * K].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g_tot = sum(ev[2 * s].elapsed_time(ev[2 * s + 1]) for s in range(K))
    p_tot = sum(ev[2 * s + 1].elapsed_time(ev[2 * s + 2]) for s in range(K))
    gmm_ms = g_tot / max(1, K * g_launches)
    pbas_ms = p_tot / max(1, K * p_launches)
    g_per = n_g / g_launches if g_launches else 0     # models per launch
    p_per = n_p / p_launches if p_launches else 0

    # Untimed: plain streaming copy of the same footprint, to calibrate what a simple
    # kernel reaches on this device.
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        fgs.fgs_copy_probe(a.data_ptr(), b.data_ptr(), nbytes, stream.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        fgs.fgs_copy_probe(a.data_ptr(), b.data_ptr(), nbytes, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b

    wall = t1 - t0
    npx = H * W
    frames_cfg = {"timed_frames": [base, base + K - 1], "untimed_frames": base,
                  "frame_sequence": "non-repeating frames of the 1280x720 sequence; at step t model j "
                                    "takes frame t + j"}
    value = L * npx * K / wall / 1e6
    g_b, p_b = gmm_bytes_per_px(), pbas_bytes_per_px()
    g_gbs = g_per * g_b * npx / (gmm_ms * 1e-3) / 1e9 if n_g else 0.0
    p_gbs = p_per * p_b * npx / (pbas_ms * 1e-3) / 1e9 if n_p else 0.0
    if S > 1:
        # kernels of different models overlap: the roofline describes a whole step (all
        # models' algorithmic bytes over the step's wall time); traffic adds the profiled
        # HBM bytes per model-frame of each kernel, which do not depend on the overlap
        step_alg = (n_g * g_b + n_p * p_b) * npx
        step_gbs = step_alg / (wall / K) / 1e9
        tg = measured_traffic_per_model("gmm_step_1280x720_k5.txt")
        tp = measured_traffic_per_model("pbas_step_1280x720_n35.txt")
        out = {
            "metric": "Mpixel-frames/s (GMM K=5 + PBAS N=35 RGB-D steps) and HBM roofline fraction",
            "value": round(value, 2), "unit": "Mpixel-frames/s", "n_gpus": 1, "steps": K,
            "warmup": args.warmup, "ms_per_step": round(wall / K * 1e3, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"RGB-D 1280x720, {n_g} GMM Kc=Kd=5 + {n_p} PBAS N=35 independent models "
                                   + ("one launch per kind and step, GMM and PBAS on their own streams"
                                      if batched else f"on {S} streams, one launch per model and step")
                                   + ", 8 moving objects + shadows",
                       "H": H, "W": W, "gmm_K": KC, "pbas_N": N_PBAS, "gmm_models": n_g, "pbas_models": n_p,
                       "streams": S, "live_state_bytes": live, **frames_cfg, "parallelism": "single GPU"},
            "roofline": {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                         "traffic": round(n_g * tg + n_p * tp) if (tg is not None and tp is not None) else None,
                         "kernel": "whole step (overlapping kernels)", "algorithmic_bytes_per_launch": step_alg},
            "copy_probe_GBs": round(copy_gbs, 1),
        }
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(rgb_h, dep_h, args.cpu_procs)
        for m, _ in models:
            m.close()
        print(json.dumps(out), flush=True)
        return
    # dominant kernel: the larger share of a step's time
    dom = "pbas" if p_launches * pbas_ms >= g_launches * gmm_ms else "gmm"
    ach = p_gbs if dom == "pbas" else g_gbs
    out = {
        "metric": "Mpixel-frames/s (GMM K=5 + PBAS N=35 RGB-D steps) and HBM roofline fraction",
        "value": round(value, 2),
        "unit": "Mpixel-frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"RGB-D 1280x720, {n_g} GMM Kc=Kd=5 + {n_p} PBAS N=35 independent models, "
                               + ("one launch per kind and step" if batched else "one launch per model and step")
                               + ", 8 moving objects + shadows",
                   "H": H, "W": W, "gmm_K": KC, "pbas_N": N_PBAS, "gmm_models": n_g, "pbas_models": n_p,
                   "live_state_bytes": live, **frames_cfg, "parallelism": "single GPU"},
        "roofline": roofline_entry(dom, pbas_ms if dom == "pbas" else gmm_ms, ach,
                                   p_per if dom == "pbas" else g_per, p_b if dom == "pbas" else g_b),
        "kernels": {k: v for k, v in (
            ("gmm_step", kernel_entry(gmm_ms, g_b, g_gbs, "gmm_step_1280x720_k5.txt", g_launches, g_per, wall / K)),
            ("pbas_step", kernel_entry(pbas_ms, p_b, p_gbs, "pbas_step_1280x720_n35.txt", p_launches, p_per,
                                       wall / K)))
            if v is not None},
        "copy_probe_GBs": round(copy_gbs, 1),
    }
    for m, _ in models:
        m.close()
    del rgb, dep
    if not args.no_serving:
        out["serving"] = serving_run(1.0, args.serve_seconds)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(rgb_h, dep_h, args.cpu_procs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
