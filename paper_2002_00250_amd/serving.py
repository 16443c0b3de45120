"""Python side of the multi-stream server (fgs_server_*): a thin wrapper and a camera-load
driver that submits frames at their arrival times (fixed frame period, random phase per
stream, uniform jitter) and collects masks and latencies.  All per-frame work runs in the
library; this module only times submissions and gathers results."""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import fgs


class Server:
    def __init__(self, hbm_budget_bytes: int, max_streams: int = 64):
        fgs.lib()
        self.handle = fgs.fgs_server_create(hbm_budget_bytes, max_streams)
        self.shapes = {}

    def open(self, algo: int, H: int, W: int, params=None) -> int:
        sid = fgs.fgs_server_open(self.handle, algo, H, W, params)
        self.shapes[sid] = (H, W)
        return sid

    def submit(self, sid: int, rgb: np.ndarray, depth: np.ndarray, t_arrival: float = 0.0) -> int:
        return fgs.fgs_server_submit(self.handle, sid, rgb.ctypes.data, depth.ctypes.data, t_arrival)

    def wait(self, ticket: int, mask: np.ndarray | None = None, timeout_ms: int = -1) -> float:
        return fgs.fgs_server_wait(self.handle, ticket, mask.ctypes.data if mask is not None else None,
                                   timeout_ms)

    def close_stream(self, sid: int) -> None:
        fgs.fgs_server_close(self.handle, sid)

    def stats(self) -> dict:
        return fgs.fgs_server_get_stats(self.handle)

    def reset_stats(self) -> None:
        fgs.fgs_server_reset_stats(self.handle)

    def destroy(self) -> None:
        if getattr(self, "handle", None):
            fgs.fgs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


@dataclass
class StreamLoad:
    sid: int
    frames: list            # [(rgb u8 [H,W,3], depth u16 [H,W]), ...], cycled
    keep_masks: bool = False
    masks: list = field(default_factory=list)
    latencies: list = field(default_factory=list)


def run_camera_load(server: Server, loads: list, duration_s: float, fps: float = 30.0,
                    jitter_s: float = 0.005, seed: int = 0):
    """Submit every stream's frames at period 1/fps from a random phase with uniform jitter,
    for duration_s seconds, from one submitting thread; one collector thread waits for the
    tickets in submission order.  Returns (per-frame latencies, wall seconds)."""
    rng = np.random.default_rng(seed)
    period = 1.0 / fps
    events = []
    for ld in loads:
        phase = rng.uniform(0.0, period)
        n = int(duration_s * fps)
        for i in range(n):
            events.append((phase + i * period + rng.uniform(-jitter_s, jitter_s), i, ld))
    events.sort(key=lambda e: e[0])
    pending = []
    cv = threading.Condition()
    done_submitting = [False]
    errors = []

    def collect():
        while True:
            with cv:
                while not pending and not done_submitting[0]:
                    cv.wait()
                if not pending:
                    return
                ticket, ld, idx = pending.pop(0)
            H, W = server.shapes[ld.sid]
            mask = np.empty((H, W), np.uint8) if ld.keep_masks else None
            try:
                lat = server.wait(ticket, mask)
            except fgs.FgsError as e:
                errors.append(e)
                continue
            ld.latencies.append(lat)
            if ld.keep_masks:
                ld.masks.append((idx, mask))

    th = threading.Thread(target=collect, daemon=True)
    th.start()
    t0 = fgs.fgs_server_now() + 0.05
    for t_rel, idx, ld in events:
        t_arr = t0 + t_rel
        dt = t_arr - fgs.fgs_server_now()
        if dt > 0:
            time.sleep(dt)
        rgb, dep = ld.frames[idx % len(ld.frames)]
        while True:
            try:
                ticket = server.submit(ld.sid, rgb, dep, t_arr)
                break
            except fgs.FgsError as e:
                if e.status != fgs.FGS_ERR_BUSY:
                    raise
                time.sleep(0.0005)
        with cv:
            pending.append((ticket, ld, idx))
            cv.notify()
    with cv:
        done_submitting[0] = True
        cv.notify()
    th.join()
    wall = fgs.fgs_server_now() - t0
    if errors:
        raise errors[0]
    lat = np.array([x for ld in loads for x in ld.latencies])
    return lat, wall
