"""Oracle trajectories for the long GPU parity runs, each in a child process.

Test infrastructure: this file runs the CPU oracle (``oracle``) on frames from the scene
generator (``synth``) and nothing else; it never loads the HIP library.

    python tests/oracle_runs.py <job.json> <out.npz>

steps one oracle model from frame 0 over ``frames`` frames of a seeded scene, restricted
to a window of the image, and saves every frame's mask over the job's ``own`` rectangle
(bit-packed) and the final state there.

Windows.  A GMM pixel's recursion involves that pixel alone (Sec. 3.1), so a window of
the image is exactly the whole image's model there.  A PBAS window draws the whole
image's random numbers (the oracle's ``origin``: counters keyed by the image's pixel
index) but misses the neighbour writes sent in from outside it (Sec. 3.2); their effect
moves at most one pixel further in per updating frame, so after u updating frames the
window agrees with the whole image at least u pixels from its inner edges (pinned on
the CPU by test_oracle_pbas.py).  ``windows()`` cuts the image into owned rectangles
that partition it and widens each by that margin on its inner sides; a pixel-frame is
then compared exactly once, against the window that owns it.

``OracleRuns`` starts the jobs as child processes (at most ``procs`` at a time) from
threads of the calling process, so the oracle runs while the caller drives the GPU.
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _split(n: int, parts: int):
    edges = [round(i * n / parts) for i in range(parts + 1)]
    return [(edges[i], edges[i + 1]) for i in range(parts)]


def windows(H: int, W: int, rows: int, cols: int, margin: int):
    """[(window (y0, x0, h, w), own (y0, x0, h, w))]: rows x cols owned rectangles
    partitioning the H x W image, each window its rectangle widened by `margin` on every
    side that is not an image border."""
    out = []
    for a, b in _split(H, rows):
        for c, d in _split(W, cols):
            y0, y1 = max(0, a - margin), min(H, b + margin)
            x0, x1 = max(0, c - margin), min(W, d + margin)
            out.append(((y0, x0, y1 - y0, x1 - x0), (a, c, b - a, d - c)))
    return out


def make_job(kind: str, scene: str, overrides: dict, params: dict, frames: int, H: int, W: int,
             window, own, frame_ids=None) -> dict:
    """`frame_ids`: the scene frame pushed at each step (default 0, 1, ..., frames - 1)."""
    ids = list(range(frames)) if frame_ids is None else [int(i) for i in frame_ids]
    assert len(ids) == frames
    return dict(kind=kind, scene=scene, overrides=overrides, params=params, frames=frames, H=H, W=W,
                window=list(window), own=list(own), frame_ids=ids)


def run(job: dict) -> dict:
    """The oracle's trajectory of one job (see the module docstring)."""
    from oracle.gmm import GmmParams, GmmRef
    from oracle.pbas import PbasParams, PbasRef
    from synth import Scene, preset

    sc = Scene(preset(job["scene"], **job["overrides"]))
    assert (sc.cfg.H, sc.cfg.W) == (job["H"], job["W"])
    y0, x0, h, w = job["window"]
    oy, ox, oh, ow = job["own"]
    ry, rx = oy - y0, ox - x0                       # own rectangle inside the window
    assert 0 <= ry and ry + oh <= h and 0 <= rx and rx + ow <= w
    prm = dict(job["params"])
    if job["kind"] == "gmm":
        ref = GmmRef(h, w, GmmParams(**prm))
    else:
        if "R_lower" in prm:
            prm["R_lower"] = tuple(prm["R_lower"])
        ref = PbasRef(h, w, PbasParams(**prm), origin=(y0, x0, job["W"]))
    masks = []
    cache = {}
    for t in job["frame_ids"]:
        if t not in cache:
            cache = {t: sc.frame(t)}
        rgb, D, _ = cache[t]
        m = ref.step(rgb[y0:y0 + h, x0:x0 + w], D[y0:y0 + h, x0:x0 + w])
        masks.append(np.packbits(m[ry:ry + oh, rx:rx + ow] != 0))
    out = {"masks": np.stack(masks)}
    for k, v in ref.state_planes().items():
        if k != "t":
            out["state_" + k] = np.ascontiguousarray(v[..., ry:ry + oh, rx:rx + ow])
    return out


class OracleRuns:
    """Runs jobs in child processes; ``result(i)`` waits for job i and loads it."""

    def __init__(self, jobs, workdir: str, procs: int | None = None):
        self.jobs = list(jobs)
        self.dir = workdir
        os.makedirs(workdir, exist_ok=True)
        procs = procs or min(16, os.cpu_count() or 1)
        self.pool = ThreadPoolExecutor(max_workers=max(1, min(procs, len(self.jobs))))
        self.lock = threading.Lock()
        self.futs = [self.pool.submit(self._one, i) for i in range(len(self.jobs))]

    def _one(self, i: int) -> str:
        jp = os.path.join(self.dir, f"job{i}.json")
        op = os.path.join(self.dir, f"job{i}.npz")
        with open(jp, "w") as f:
            json.dump(self.jobs[i], f)
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), jp, op], env=env,
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"oracle job {i} failed ({r.returncode}): {r.stderr[-2000:]}")
        return op

    def result(self, i: int) -> dict:
        path = self.futs[i].result()
        with np.load(path) as z:
            return {k: z[k] for k in z.files}

    def close(self):
        self.pool.shutdown(wait=True, cancel_futures=True)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    with open(sys.argv[1]) as f:
        job = json.load(f)
    res = run(job)
    np.savez(sys.argv[2], **res)
