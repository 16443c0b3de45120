"""Multi-stream server: every stream's masks in the batched mix are identical to the
oracle's run of that stream and to the same stream driven alone through fgs_push_frame;
admission by HBM budget; back-pressure; close with frames queued; the 32-stream, 30 fps
mixed-resolution workload within one frame period at p99, three of its streams compared
with the oracle over every served frame."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import log  # noqa: E402
from oracle.gmm import GmmParams, GmmRef  # noqa: E402
from oracle.pbas import PbasParams, PbasRef  # noqa: E402
from oracle_runs import OracleRuns, make_job, windows  # noqa: E402
from synth import Scene, preset  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


def _params(algo, K=5, N=20, seed=None, gmm_variant=False):
    from paper_2002_00250_amd import fgs
    if algo == fgs.FGS_GMM:
        p = fgs.fgs_gmm_params_default()
        p.Kc = p.Kd = K
        if gmm_variant:                   # rate alpha / w and the density decision
            p.rho_mode, p.decision = 1, 1
    else:
        p = fgs.fgs_pbas_params_default()
        p.N = N
        if seed is not None:
            p.seed = seed
    return p


def _frames(H, W, n, seed):
    sc = Scene(preset("pbas_640x480", H=H, W=W, seed=seed))
    return [sc.frame(t)[:2] for t in range(n)]


def _oracle_params(algo, p):
    """The oracle's constants for a stream opened with the library's params `p` (the
    library's defaults are the oracle's; only the fields these tests change are copied)."""
    from paper_2002_00250_amd import fgs
    if algo == fgs.FGS_GMM:
        return GmmParams(Kc=p.Kc, Kd=p.Kd, rho_mode=p.rho_mode, decision=p.decision, var_mode=p.var_mode)
    return PbasParams(N=p.N, seed=p.seed, gradient=bool(p.gradient), grad_alpha=p.grad_alpha)


def _oracle(algo, H, W, params, frames):
    """The oracle's masks for a stream's frames, from frame 0."""
    from paper_2002_00250_amd import fgs
    op = _oracle_params(algo, params)
    ref = GmmRef(H, W, op) if algo == fgs.FGS_GMM else PbasRef(H, W, op)
    return [ref.step(rgb, dep) for rgb, dep in frames]


def _alone(algo, H, W, params, frames):
    from paper_2002_00250_amd import fgs
    m = fgs.Model(algo, H, W, params)
    out = []
    for rgb, dep in frames:
        m.push(rgb, dep)
        out.append(m.mask_host())
    m.close()
    return out


@pytest.mark.parametrize("gmm_variant", [False, True])
def test_mix_equals_alone(gmm_variant):
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server
    specs = [(fgs.FGS_GMM, 48, 64), (fgs.FGS_PBAS, 48, 64), (fgs.FGS_GMM, 70, 100),
             (fgs.FGS_PBAS, 70, 100), (fgs.FGS_GMM, 120, 160), (fgs.FGS_PBAS, 121, 159),
             (fgs.FGS_PBAS, 5, 7)]
    T = 36
    srv = Server(1 << 30, 16)
    streams = []
    for i, (algo, H, W) in enumerate(specs):
        p = _params(algo, seed=1000 + i, gmm_variant=gmm_variant)
        streams.append((srv.open(algo, H, W, p), algo, H, W, p, _frames(H, W, T, seed=50 + i)))
    got = {sid: [] for sid, *_ in streams}
    for t in range(T):
        tickets = []
        for sid, algo, H, W, p, fr in streams:
            if (t + sid) % 3 == 0 and t > 0:      # uneven arrivals: batches of different make-up
                continue
            tickets.append((sid, srv.submit(sid, *fr[t]), H, W))
        for sid, tk, H, W in tickets:
            m = np.empty((H, W), np.uint8)
            srv.wait(tk, m)
            got[sid].append(m)
        for sid, algo, H, W, p, fr in streams:   # the skipped ones now
            if (t + sid) % 3 == 0 and t > 0:
                m = np.empty((H, W), np.uint8)
                srv.wait(srv.submit(sid, *fr[t]), m)
                got[sid].append(m)
    st = srv.stats()
    log(f"server mix: {st['frames_done']} frames in {st['batches']} batches "
        f"({st['mean_batch_frames']:.2f} per batch)")
    for sid, algo, H, W, p, fr in streams:
        ref = _alone(algo, H, W, p, fr)
        orc = _oracle(algo, H, W, p, fr)
        diff = sum(int((a != b).sum()) for a, b in zip(got[sid], ref))
        odiff = sum(int((a != b).sum()) for a, b in zip(got[sid], orc))
        log(f"stream {sid} ({'GMM' if algo == fgs.FGS_GMM else 'PBAS'} {H}x{W}): {odiff} mask pixels "
            f"differ from the oracle, {diff} from the stream alone")
        assert len(got[sid]) == T and odiff == 0 and diff == 0
    srv.destroy()


def test_pbas_n_up_to_40_in_the_mix_equals_alone():
    # the server's PBAS instance covers N <= 40 with run-time bounds on every quad of
    # slots: N = 35 (one padding slot) and N = 5 next to each other in one launch
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server
    srv = Server(1 << 30, 8)
    specs = [(fgs.FGS_PBAS, 70, 100, 35), (fgs.FGS_PBAS, 33, 47, 5), (fgs.FGS_GMM, 40, 64, 0)]
    T = 45
    streams = []
    for i, (algo, H, W, N) in enumerate(specs):
        p = _params(algo, K=3, N=max(N, 2), seed=77 + i)
        streams.append((srv.open(algo, H, W, p), algo, H, W, p, _frames(H, W, T, seed=90 + i)))
    got = {sid: [] for sid, *_ in streams}
    for t in range(T):
        tickets = [(sid, srv.submit(sid, *fr[t]), H, W) for sid, algo, H, W, p, fr in streams]
        for sid, tk, H, W in tickets:
            m = np.empty((H, W), np.uint8)
            srv.wait(tk, m)
            got[sid].append(m)
    for sid, algo, H, W, p, fr in streams:
        ref = _alone(algo, H, W, p, fr)
        orc = _oracle(algo, H, W, p, fr)
        diff = sum(int((a != b).sum()) for a, b in zip(got[sid], ref))
        odiff = sum(int((a != b).sum()) for a, b in zip(got[sid], orc))
        log(f"server N<=40 mix: stream {sid} ({'GMM' if algo == fgs.FGS_GMM else 'PBAS N=%d' % p.N} {H}x{W}): "
            f"{odiff} mask pixels differ from the oracle, {diff} from alone")
        assert odiff == 0 and diff == 0
    srv.destroy()


def test_admission_by_budget_and_close():
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server
    srv = Server(64 << 20, 8)
    ids = []
    with pytest.raises(fgs.FgsError) as e:
        for _ in range(10):
            ids.append(srv.open(fgs.FGS_GMM, 240, 320, _params(fgs.FGS_GMM)))
    assert e.value.status == fgs.FGS_ERR_BUSY and len(ids) >= 1
    used = srv.stats()["device_bytes_used"]
    assert used <= 64 << 20
    srv.close_stream(ids[0])
    assert srv.stats()["device_bytes_used"] < used
    ids[0] = srv.open(fgs.FGS_GMM, 240, 320, _params(fgs.FGS_GMM))   # admitted again
    bad = _params(fgs.FGS_GMM)
    bad.Kc, bad.Kd = 4, 2                                           # no such model
    with pytest.raises(fgs.FgsError) as e:
        srv.open(fgs.FGS_GMM, 24, 32, bad)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    srv.destroy()


def test_every_stream_class_in_one_server():
    # One server, streams of every kernel class: GMM K = 5 and K = 3 (both eligible for the
    # fused serving launch; the one with fewer pixels runs in the step kernels), the
    # paper's 7/3, K = 1, per-channel variances, the rate and decision variants; PBAS
    # N = 20 and 35 (fused), 50 and 64 (step kernels), 5, and the gradient-magnitude
    # variant (a launch of its own).  Uneven arrivals make batches
    # of changing make-up.  Every stream equals the oracle and the stream alone.
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server
    G, P = fgs.FGS_GMM, fgs.FGS_PBAS
    specs = [(G, 40, 64, dict(K=(5, 5))), (G, 33, 47, dict(K=(3, 3))), (G, 30, 70, dict(K=(7, 3))),
             (G, 21, 37, dict(K=(1, 1))), (G, 45, 60, dict(K=(5, 5), var_mode=1)),
             (G, 28, 50, dict(K=(3, 3), rho_mode=2, decision=1)), (G, 64, 80, dict(K=(5, 5), rho_mode=1)),
             (P, 36, 70, dict(N=20)), (P, 29, 66, dict(N=35)), (P, 24, 40, dict(N=50)),
             (P, 17, 65, dict(N=64)), (P, 9, 10, dict(N=5)), (P, 23, 45, dict(N=10, gradient=1))]
    T = 72
    srv = Server(1 << 30, 16)
    streams = []
    for i, (algo, H, W, o) in enumerate(specs):
        if algo == G:
            p = fgs.fgs_gmm_params_default()
            p.Kc, p.Kd = o["K"]
            p.var_mode, p.rho_mode, p.decision = o.get("var_mode", 0), o.get("rho_mode", 0), o.get("decision", 0)
        else:
            p = fgs.fgs_pbas_params_default()
            p.N, p.seed, p.gradient = o["N"], 4000 + i, o.get("gradient", 0)
        streams.append((srv.open(algo, H, W, p), algo, H, W, p, _frames(H, W, T, seed=500 + i)))
    got = {sid: [] for sid, *_ in streams}
    for t in range(T):
        late = [st for st in streams if (t * 7 + st[0]) % 4 == 0 and t > 0]
        tickets = [(sid, srv.submit(sid, *fr[t]), H, W) for sid, algo, H, W, p, fr in streams
                   if not ((t * 7 + sid) % 4 == 0 and t > 0)]
        for sid, tk, H, W in tickets:
            m = np.empty((H, W), np.uint8)
            srv.wait(tk, m)
            got[sid].append(m)
        for sid, algo, H, W, p, fr in late:
            m = np.empty((H, W), np.uint8)
            srv.wait(srv.submit(sid, *fr[t]), m)
            got[sid].append(m)
    st = srv.stats()
    log(f"every class: {st['frames_done']} frames in {st['batches']} batches")
    for sid, algo, H, W, p, fr in streams:
        orc = _oracle(algo, H, W, p, fr)
        ref = _alone(algo, H, W, p, fr)
        odiff = sum(int((a != b).sum()) for a, b in zip(got[sid], orc))
        diff = sum(int((a != b).sum()) for a, b in zip(got[sid], ref))
        what = (f"GMM {p.Kc}/{p.Kd} var {p.var_mode} rho {p.rho_mode} dec {p.decision}" if algo == G
                else f"PBAS N={p.N}" + (" gradient" if p.gradient else ""))
        fg = sum(int((m != 0).sum()) for m in got[sid])
        log(f"stream {sid} ({what}, {H}x{W}): {odiff} mask pixels differ from the oracle, {diff} from alone "
            f"({fg} foreground pixel-frames)")
        assert len(got[sid]) == T and odiff == 0 and diff == 0
    srv.destroy()


def test_backpressure_and_close_with_frames_queued():
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server
    srv = Server(1 << 30, 4)
    sid = srv.open(fgs.FGS_PBAS, 64, 96, _params(fgs.FGS_PBAS))
    fr = _frames(64, 96, 6, seed=3)
    tickets = [srv.submit(sid, *fr[i]) for i in range(4)]
    with pytest.raises(fgs.FgsError) as e:
        srv.submit(sid, *fr[4])                     # ring of 4 full until collected
    assert e.value.status == fgs.FGS_ERR_BUSY
    srv.wait(tickets[0])
    t5 = srv.submit(sid, *fr[4])
    srv.close_stream(sid)
    outcomes = []
    for tk in tickets[1:] + [t5]:
        try:
            srv.wait(tk, timeout_ms=10000)
            outcomes.append("done")
        except fgs.FgsError as err:
            assert err.status == fgs.FGS_ERR_BAD_STATE
            outcomes.append("dropped")
    log(f"close with frames queued: {outcomes}")
    with pytest.raises(fgs.FgsError):
        srv.submit(sid, *fr[5])
    srv.destroy()


def test_close_during_submit_never_strands_a_ticket():
    # close_stream racing a submit whose frame copy is under way: the ticket must end as
    # done or dropped (never left queued on a closed stream, where a wait would not return)
    import threading
    import time
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server
    H, W = 720, 1280
    rgb = np.zeros((H, W, 3), np.uint8)
    dep = np.full((H, W), 1500, np.uint16)
    outcomes = {"done": 0, "dropped": 0, "refused": 0}
    for rnd in range(4):
        srv = Server(8 << 30, 4)
        for i in range(30):
            sid = srv.open(fgs.FGS_GMM, H, W, _params(fgs.FGS_GMM))
            box = {}

            def sub():
                try:
                    box["t"] = srv.submit(sid, rgb, dep)
                except fgs.FgsError as err:
                    box["err"] = err.status
            th = threading.Thread(target=sub)
            th.start()
            time.sleep(1e-4 * (i % 8))
            srv.close_stream(sid)
            th.join()
            if "t" in box:
                try:
                    srv.wait(box["t"], timeout_ms=5000)
                    outcomes["done"] += 1
                except fgs.FgsError as err:
                    assert err.status == fgs.FGS_ERR_BAD_STATE, err.status   # BUSY: stranded
                    outcomes["dropped"] += 1
            else:
                assert box["err"] == fgs.FGS_ERR_INVALID_ARG
                outcomes["refused"] += 1
        srv.destroy()
    log(f"close during submit: {outcomes}")


def test_concurrent_opens_respect_max_streams():
    # opens racing each other: the server admits exactly max_streams of them (its batch
    # descriptors hold max_streams entries), refuses the rest as BUSY, and admits again
    # after a close
    import threading
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server
    for rnd in range(3):
        srv = Server(1 << 30, 3)
        gate = threading.Barrier(8)
        got = {"ok": [], "busy": 0}
        lock = threading.Lock()

        def opener(j):
            gate.wait()
            try:
                sid = srv.open(fgs.FGS_GMM if j % 2 else fgs.FGS_PBAS, 48, 64,
                               _params(fgs.FGS_GMM if j % 2 else fgs.FGS_PBAS))
                with lock:
                    got["ok"].append(sid)
            except fgs.FgsError as err:
                assert err.status == fgs.FGS_ERR_BUSY, err.status
                with lock:
                    got["busy"] += 1
        ths = [threading.Thread(target=opener, args=(j,)) for j in range(8)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        assert len(got["ok"]) == 3 and got["busy"] == 5, got
        assert srv.stats()["streams_open"] == 3
        fr = _frames(48, 64, 2, seed=rnd)
        for sid in got["ok"]:                       # every admitted stream serves a frame
            srv.wait(srv.submit(sid, *fr[0]), timeout_ms=10000)
        srv.close_stream(got["ok"][0])
        srv.open(fgs.FGS_GMM, 48, 64, _params(fgs.FGS_GMM))
        with pytest.raises(fgs.FgsError) as e:
            srv.open(fgs.FGS_GMM, 48, 64, _params(fgs.FGS_GMM))
        assert e.value.status == fgs.FGS_ERR_BUSY
        srv.destroy()


def test_ticket_collected_once_and_closed_streams_released():
    # a ticket is collected by one wait; a second wait (after it, or racing it) reports an
    # unknown ticket instead of touching a released stream; streams closed with frames
    # pending are released once their tickets are collected, over many open/close cycles
    import threading
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server
    srv = Server(1 << 30, 4)
    fr = _frames(48, 64, 3, seed=9)
    sid = srv.open(fgs.FGS_PBAS, 48, 64, _params(fgs.FGS_PBAS))
    tk = srv.submit(sid, *fr[0])
    srv.wait(tk, timeout_ms=10000)
    with pytest.raises(fgs.FgsError) as e:
        srv.wait(tk, timeout_ms=100)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    for cycle in range(40):
        sid2 = srv.open(fgs.FGS_GMM, 48, 64, _params(fgs.FGS_GMM))
        tks = [srv.submit(sid2, *fr[i]) for i in range(3)]
        res = {"ok": 0, "other": []}
        lock = threading.Lock()

        def waiter(t):
            try:
                srv.wait(t, timeout_ms=10000)
                with lock:
                    res["ok"] += 1
            except fgs.FgsError as err:
                with lock:
                    res["other"].append(err.status)
        ths = [threading.Thread(target=waiter, args=(tks[0],)) for _ in range(2)]
        for t in ths:
            t.start()
        srv.close_stream(sid2)
        for t in ths:
            t.join()
        # the first frame is done or dropped: one wait collects it, the other finds it gone
        assert res["ok"] + res["other"].count(fgs.FGS_ERR_BAD_STATE) == 1, res
        assert res["other"].count(fgs.FGS_ERR_INVALID_ARG) == 1, res
        for t in tks[1:]:
            try:
                srv.wait(t, timeout_ms=10000)
            except fgs.FgsError as err:
                assert err.status == fgs.FGS_ERR_BAD_STATE, err.status
    assert srv.stats()["streams_open"] == 1
    srv.wait(srv.submit(sid, *fr[1]), timeout_ms=10000)
    bad = fgs.fgs_pbas_params_default()
    bad.struct_size = 8                                   # wrong struct size: refused, nothing read
    with pytest.raises(fgs.FgsError) as e:
        srv.open(fgs.FGS_PBAS, 48, 64, bad)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    srv.destroy()


def test_32_streams_30fps_mixed_resolution():
    # 12x 424x240, 12x 640x480, 8x 1280x720; even streams GMM K=5, odd PBAS N=20;
    # frames at 30 fps, random phase, +-5 ms jitter.  p99 latency below one frame period,
    # and three streams' masks identical to the same streams alone.
    from paper_2002_00250_amd import fgs
    from paper_2002_00250_amd.serving import Server, StreamLoad, run_camera_load
    sizes = [(240, 424)] * 12 + [(480, 640)] * 12 + [(720, 1280)] * 8
    srv = Server(64 << 30, 32)
    loads, meta = [], []
    for i, (H, W) in enumerate(sizes):
        algo = fgs.FGS_GMM if i % 2 == 0 else fgs.FGS_PBAS
        p = _params(algo, seed=7000 + i)
        sid = srv.open(algo, H, W, p)
        fr = _frames(H, W, 4, seed=300 + i)
        keep = i in (0, 13, 31)
        loads.append(StreamLoad(sid, fr, keep_masks=keep))
        meta.append((algo, H, W, p))
    warm = [StreamLoad(ld.sid, ld.frames) for ld in loads]
    run_camera_load(srv, warm, duration_s=1.0, seed=1)       # PBAS fills its samples
    srv.reset_stats()
    lat, wall = run_camera_load(srv, loads, duration_s=3.0, seed=2)
    st = srv.stats()
    p50, p99 = np.percentile(lat, 50), np.percentile(lat, 99)
    offered = sum(H * W for H, W in sizes) * 30 / 1e6
    log(f"32 streams @30fps: {lat.size} frames, p50 {p50 * 1e3:.2f} ms, p99 {p99 * 1e3:.2f} ms, "
        f"max {lat.max() * 1e3:.2f} ms; {st['mean_batch_frames']:.2f} frames/batch; "
        f"{st['mpix_frames_per_s']:.1f} Mpx-f/s served (offered {offered:.1f})")
    assert p99 < 1.0 / 30
    # masks of three streams equal the oracle's run and the same frames pushed alone
    # (warm-up frames first); the served frames cycle through 4 scene frames, counted from
    # 0 again in the measured run.  The oracle follows the two PBAS streams in windows
    # with the neighbour updates' propagation margin, in child processes.
    kept = (0, 13, 31)
    jobs, owner = [], {}
    for i in kept:
        algo, H, W, p = meta[i]
        nw, nl = len(warm[i].latencies), len(loads[i].latencies)
        ids = [k % 4 for k in range(nw)] + [k % 4 for k in range(nl)]
        kind = "gmm" if algo == fgs.FGS_GMM else "pbas"
        op = _oracle_params(algo, p)
        prm = dict(Kc=op.Kc, Kd=op.Kd) if kind == "gmm" else dict(N=op.N, seed=op.seed)
        grid = (1, 1) if kind == "gmm" else ((2, 4) if H >= 720 else (1, 2))
        margin = 0 if kind == "gmm" else max(0, len(ids) - op.N)
        owner[i] = []
        for win, own in windows(H, W, *grid, margin):
            owner[i].append(len(jobs))
            jobs.append(make_job(kind, "pbas_640x480", dict(H=H, W=W, seed=300 + i), prm, len(ids), H, W,
                                 win, own, frame_ids=ids))
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        runs = OracleRuns(jobs, td)
        try:
            for i in kept:
                algo, H, W, p = meta[i]
                seq = [loads[i].frames[k % 4] for k in range(len(warm[i].latencies))] + \
                      [loads[i].frames[k % 4] for k in range(len(loads[i].latencies))]
                nw = len(warm[i].latencies)
                ref = _alone(algo, H, W, p, seq)[nw:]
                got = [m for _, m in sorted(loads[i].masks, key=lambda x: x[0])]
                diff = sum(int((a != b).sum()) for a, b in zip(got, ref))
                exp = np.zeros((len(seq), H, W), bool)
                for j in owner[i]:
                    oy, ox, oh, ow = jobs[j]["own"]
                    mk = runs.result(j)["masks"]
                    exp[:, oy:oy + oh, ox:ox + ow] = np.unpackbits(mk, axis=1)[:, :oh * ow].reshape(
                        len(seq), oh, ow).astype(bool)
                odiff = sum(int(((a != 0) != b).sum()) for a, b in zip(got, exp[nw:]))
                log(f"stream {i} ({'GMM' if algo == fgs.FGS_GMM else 'PBAS'} {H}x{W}): over {len(got)} served "
                    f"frames (after {nw} warm-up frames) {odiff} mask pixels differ from the oracle, "
                    f"{diff} from alone")
                assert len(got) == len(ref) and odiff == 0 and diff == 0
        finally:
            runs.close()
    srv.destroy()
