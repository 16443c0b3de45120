"""Sector-granular HBM traffic floor of one PBAS step, counted from the oracle's own run.

The step kernel keeps the PBAS state in slot-major planes (samples as 16-byte quads of
four slots per pixel, the D history as one 32-bit word of four channel bytes per slot and
pixel, R and T as float4, S as four uint16, the pixel's previous value in the first
padding slot for N >= 33 not a multiple of 4).  DRAM moves whole sectors, so what a frame
must move is counted here per sector of `gran` bytes:

reads   every sample quad (the classification compares all N slots), T, S, the RGB
        and depth input, the fire bytes of the tile and its 1-pixel halo (64 x 4 tiles),
        R where some channel's R is off its lower bound (the fire byte flags the pixels
        whose four R values sit on it), and each D-history sector holding the old byte of
        a self-update (Sec. 3.2: the update replaces D_k with d_min, and the running sum S
        needs the value it drops);
writes  each sample-quad sector in which some byte changes, plus the quad holding the
        previous-value slot (rewritten every frame), each D sector with a changed byte,
        each R / T / S sector with a changed value, the mask and the fire bytes.

A pixel's state is its own, so a sector's bytes belong to consecutive pixels of one row
(16 pixels per 64-byte D sector, 4 per sample-quad or R/T sector, 8 per S sector); the
image width must be a multiple of gran / 4 pixels.  The counts use the oracle's state
before and after each frame and its Philox words for the self-update slots
(``PbasRef.last_draws``, ``last_self``); nothing here touches the GPU path.

    python tests/pbas_traffic_floor.py [--frames 100:106] [--every K] [--out FILE]

runs the 1280x720 N = 35 benchmark sequence from frame 0 and prints (or writes) the
per-pixel-frame averages over the given frames at 64- and 128-byte sectors, and the floor
at the request sizes of the device (reads in 128-byte lines, writes in 64-byte sectors)."""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.pbas import NB_DX, NB_DY, PbasParams, PbasRef  # noqa: E402

TILE_W, TILE_H = 64, 4


def _sectors(touched: np.ndarray, px_per_sector: int) -> int:
    """Number of sectors of px_per_sector consecutive row pixels holding a True pixel."""
    H, W = touched.shape
    assert W % px_per_sector == 0, (W, px_per_sector)
    return int(touched.reshape(H, W // px_per_sector, px_per_sector).any(-1).sum())


def _plane_sectors(k, y, x, W: int, H: int, px_per_sector: int) -> int:
    """Distinct (plane k, row y, sector of x) triples among the given pixel events."""
    assert W % px_per_sector == 0, (W, px_per_sector)
    if len(k) == 0:
        return 0
    key = (np.asarray(k, np.int64) * H + np.asarray(y, np.int64)) * (W // px_per_sector) + \
        np.asarray(x, np.int64) // px_per_sector
    return int(np.unique(key).size)


def fire_halo_bytes_per_px(H: int, W: int) -> float:
    """Fire bytes a frame reads: each 64 x 4 tile reads its pixels and a 1-pixel ring
    (clipped at the image border)."""
    n = 0
    for y0 in range(0, H, TILE_H):
        for x0 in range(0, W, TILE_W):
            hy = min(H, y0 + TILE_H + 1) - max(0, y0 - 1)
            hx = min(W, x0 + TILE_W + 1) - max(0, x0 - 1)
            n += hy * hx
    return n / (H * W)


def last_in_pad(N: int) -> bool:
    return N >= 33 and N % 4 != 0


def step_traffic(ref: PbasRef, rgb: np.ndarray, depth: np.ndarray, grans=(64, 128)) -> dict:
    """Advance ``ref`` by one updating frame and return {gran: {part: bytes per pixel}}."""
    if ref.t < ref.p.N:
        raise ValueError("count updating frames only (the model is still filling)")
    H, W, N = ref.H, ref.W, ref.p.N
    S0, D0, R0, T0, Sm0 = ref.samples.copy(), ref.D.copy(), ref.R.copy(), ref.T.copy(), ref.S.copy()
    r_bound = (R0.view(np.uint32) == np.array(ref.p.R_lower, np.float32).view(np.uint32)).all(-1)
    ref.step(rgb, depth)
    w0, w1 = ref.last_draws
    kself = (((w0 & np.uint32(0xFFFF)).astype(np.uint64) * np.uint64(N)) >> np.uint64(16)).astype(np.int64)
    upd = ref.last_self                                   # [H, W, 4] self-updates this frame
    # slots an update lands in, whether or not the byte changes: the self-updates and the
    # neighbour writes (direction (w1 >> 13) & 7, slot ((w1 & 0x1FFF) * N) >> 13, into a
    # neighbour inside the image, the depth channel only where that neighbour has depth)
    ys, xs, js = np.nonzero(upd)
    ks = kself[ys, xs, js]
    self_evt = (ks, ys, xs)                            # D reads, and self-update landings
    ys, xs, js = np.nonzero(ref.last_nb)
    d = ((w1[ys, xs, js] >> np.uint32(13)) & np.uint32(7)).astype(np.int64)
    k = (((w1[ys, xs, js] & np.uint32(0x1FFF)).astype(np.uint64) * np.uint64(N)) >> np.uint64(13)).astype(np.int64)
    ny, nx = ys + NB_DY[d], xs + NB_DX[d]
    ok = (ny >= 0) & (ny < H) & (nx >= 0) & (nx < W)
    ok[ok] &= (js[ok] < 3) | (np.asarray(depth)[ny[ok], nx[ok]] > 0)
    nb_evt = (k[ok], ny[ok], nx[ok])
    land_k = np.concatenate([self_evt[0], nb_evt[0]])
    land_y = np.concatenate([self_evt[1], nb_evt[1]])
    land_x = np.concatenate([self_evt[2], nb_evt[2]])
    d_chg = np.nonzero((ref.D != D0).any(-1))                # (k, y, x) of changed D words
    s_chg = np.nonzero((ref.samples != S0).any(-1))          # (k, y, x) of changed sample words
    pad = last_in_pad(N)
    nq = (N + 3) // 4
    npx = H * W
    last_q = N // 4 if pad else None                         # quad holding the previous value
    out = {}
    for g in grans:
        dpx, qpx, spx = g // 4, g // 16, g // 8
        r = {}
        r["samples_read"] = 16.0 * nq + (0.0 if pad else 4.0)
        r["TS_read"] = 24.0
        # R is read only where some channel's R left its lower bound: the pixel's fire byte
        # carries the flags (R_lower itself stands in for it elsewhere)
        r["R_read"] = _sectors(~r_bound, qpx) * g / npx
        r["input_read"] = 5.0
        r["fire_read"] = fire_halo_bytes_per_px(H, W)
        r["D_read"] = _plane_sectors(*self_evt, W, H, dpx) * g / npx

        def quad_sectors(k, y, x):
            q = np.asarray(k) // 4
            keep = q != last_q if pad else np.ones(len(q), bool)
            n = _plane_sectors(q[keep], np.asarray(y)[keep], np.asarray(x)[keep], W, H, qpx)
            return n + (H * (W // qpx) if pad else 0)        # the previous-value quad: every sector
        r["samples_write"] = quad_sectors(*s_chg) * g / npx + (0.0 if pad else 4.0)
        landed_bytes = quad_sectors(land_k, land_y, land_x) * g / npx + (0.0 if pad else 4.0)
        r["D_write"] = _plane_sectors(*d_chg, W, H, dpx) * g / npx
        r["R_write"] = _sectors((ref.R != R0).any(-1), qpx) * g / npx
        r["T_write"] = _sectors((ref.T != T0).any(-1), qpx) * g / npx
        r["S_write"] = _sectors((ref.S != Sm0).any(-1), spx) * g / npx
        r["mask_fire_write"] = 2.0
        r["total"] = sum(r.values())
        # not part of the floor: sample sectors an update lands in (a write of an equal
        # byte included), which a kernel that does not compare bytes writes back
        r["samples_landed"] = landed_bytes
        out[g] = r
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", default="100:106", help="first:end of the counted frames")
    ap.add_argument("--every", type=int, default=1, help="count every k-th frame of the range")
    ap.add_argument("--N", type=int, default=35)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    from synth import Scene, preset
    f0, f1 = (int(v) for v in a.frames.split(":"))
    cfg = preset("hd_1280x720")
    sc = Scene(cfg)
    ref = PbasRef(cfg.H, cfg.W, PbasParams(N=a.N))
    t0 = time.time()
    for t in range(f0):
        rgb, D, _ = sc.frame(t)
        ref.step(rgb, D)
    acc = {}
    rates = {"self_update": 0.0, "neighbour": 0.0, "foreground": 0.0}
    counted = list(range(f0, f1, a.every))
    n = len(counted)
    for t in range(f0, f1):
        rgb, D, _ = sc.frame(t)
        if t not in counted:
            ref.step(rgb, D)
            continue
        res = step_traffic(ref, rgb, D)
        for g, r in res.items():
            for k, v in r.items():
                acc.setdefault(g, {}).setdefault(k, 0.0)
                acc[g][k] += v / n
        rates["self_update"] += ref.last_self.mean() / n
        rates["neighbour"] += ref.last_nb.mean() / n
        rates["foreground"] += ref.last_F.any(-1).mean() / n
    lines = [f"# PBAS N={a.N} traffic floor on the 1280x720 benchmark sequence (oracle count)", "",
             f"frames: {f0}..{f1 - 1}" + (f", every {a.every}th counted ({n} frames)" if a.every > 1 else "")
             + " (model run from frame 0)",
             f"rates per pixel-channel: self-update {rates['self_update']:.4f}, neighbour "
             f"{rates['neighbour']:.4f}; foreground pixels {rates['foreground']:.4f}"]
    reads = ("samples_read", "TS_read", "R_read", "input_read", "fire_read", "D_read")
    for g in sorted(acc):
        lines.append(f"floor_bytes_per_px_{g}: {acc[g]['total']:.1f}")
    # the device's request sizes: every read request a 128-byte line, writes 64-byte sectors
    rd = sum(acc[128][k] for k in reads)
    wr = sum(v for k, v in acc[64].items() if k not in reads + ("total", "samples_landed"))
    lines.append(f"floor_bytes_per_px: {rd + wr:.1f}")
    lines.append(f"floor_read_bytes_per_px: {rd:.1f}")
    lines.append(f"floor_write_bytes_per_px: {wr:.1f}")
    lines.append("(floor_bytes_per_px: reads counted in 128-byte lines and writes in 64-byte sectors, the "
                 "request sizes rocprofv3 reports for the step kernels on MI355X)")
    for g in sorted(acc):
        lines.append("")
        lines.append(f"{g}-byte sectors, bytes per pixel-frame (sample sectors an update lands in, "
                     f"equal bytes included: {acc[g]['samples_landed']:.2f}):")
        for k, v in acc[g].items():
            if k not in ("total", "samples_landed"):
                lines.append(f"  {k:16s} {v:8.2f}")
    lines += ["", "command:", f"  python tests/pbas_traffic_floor.py --frames {a.frames} --every {a.every} --N {a.N}"
              + (f" --out {a.out}" if a.out else ""), f"({time.time() - t0:.0f} s on the host)"]
    text = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
