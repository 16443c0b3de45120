"""bench.py --summarize-profiles on small synthetic rocprofv3 CSV files: kernel names are
shortened to their template form, durations and counters are averaged over each kernel's
last PROFILE_STEPS dispatches only, read bytes come from the request counts by size, and
the summary files carry what bench.py later reads back (traffic per launch, hash lock)."""
import csv
import os

import pytest

import bench


def test_short_kernel_names():
    f = bench._short_kernel_name
    assert f("void fgs::(anonymous namespace)::gmm_step_kernel<8, 5, 5, true, false, 1>(fgs::GmmBatch<8>)") == \
        "gmm_step_kernel<8, 5, 5, true, false, 1>"
    assert f("fgs::(anonymous namespace)::copy_kernel(HIP_vector_type<unsigned int, 4u> const*, long)") == "copy_kernel"
    assert f("__amd_rocclr_fillBufferAligned") == "__amd_rocclr_fillBufferAligned"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


KERNELS = {
    "gmm": "void fgs::(anonymous namespace)::gmm_step_kernel<8, 5, 5, true, false, 1>(fgs::GmmBatch<8>)",
    "pbas": "void fgs::(anonymous namespace)::pbas_step_kernel<8, 36, true>(fgs::PbasBatch<8>)",
    "copy": "fgs::(anonymous namespace)::copy_kernel(HIP_vector_type<unsigned int, 4u> const*, long)",
}


@pytest.fixture
def profile_dir(tmp_path, monkeypatch):
    """Each step kernel has 5 untimed dispatches (duration 900, counters x 10) before
    PROFILE_STEPS timed ones (duration 100 + 2 i for the gmm, 200 for pbas)."""
    monkeypatch.setattr(bench, "PROFILE_STEPS", 4)
    out = tmp_path / "profiles"
    out.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for src in {s for v in bench.STEP_KERNELS.values() for s in v[2]}:
        p = tmp_path / src
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_text("source " + src)
    d = tmp_path / "raw"
    disp = []
    did = 0
    for i in range(9):
        for k in ("gmm", "pbas"):
            did += 1
            timed = i >= 5
            dur = (100 + 2 * (i - 5) if k == "gmm" else 200) if timed else 900
            disp.append((did, KERNELS[k], dur, timed))
    did += 1
    disp.append((did, KERNELS["copy"], 1000, True))
    tr_header = ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    _write(str(d / "stats" / "bench_kernel_trace.csv"), tr_header,
           [["KERNEL_DISPATCH", i, n, 1000 * i, 1000 * i + dur] for i, n, dur, _ in disp])
    st_header = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"]
    rows = []
    for k, n in KERNELS.items():
        ds = [dur for _, nn, dur, _ in disp if nn == n]
        rows.append([n, len(ds), sum(ds), sum(ds) / len(ds), 0.0, min(ds), max(ds), 0.0])
    _write(str(d / "stats" / "bench_kernel_stats.csv"), st_header, rows)
    cc_header = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]

    def counters(sub, per):
        rows = []
        for i, n, _, timed in disp:
            for c, v in per(n).items():
                rows.append([i, n, c, v if (timed or n == KERNELS["copy"]) else 10 * v])
        _write(str(d / sub / "run_counter_collection.csv"), cc_header, rows)
    copy_bytes = bench.COPY_BYTES
    counters("pmc_FETCH_SIZE", lambda n: {"FETCH_SIZE": (copy_bytes / 2 if n == KERNELS["copy"] else 1000) / 1024})
    counters("pmc_WRITE_SIZE", lambda n: {"WRITE_SIZE": (copy_bytes if n == KERNELS["copy"] else 2048) / 1024})
    counters("pmc_rdreq", lambda n: {"TCC_EA0_RDREQ_32B_sum": 1, "TCC_EA0_RDREQ_64B_sum": 2,
                                     "TCC_EA0_RDREQ_128B_sum": copy_bytes / 128 if n == KERNELS["copy"] else 3})
    counters("pmc_wrreq", lambda n: {"TCC_EA0_WRREQ_sum": 7, "TCC_EA0_WRREQ_64B_sum": 5})
    return d, out


def test_summary_averages_the_timed_dispatches(profile_dir):
    d, out = profile_dir
    bench.summarize_profiles(str(d))
    kv = bench._kv(str(out / "gmm_step_1280x720_k5.txt"))
    assert float(kv["avg_duration_ns"]) == pytest.approx((100 + 102 + 104 + 106) / 4)
    assert int(kv["timed_dispatches"]) == 4
    assert float(kv["avg_duration_all_calls_ns"]) == pytest.approx((5 * 900 + 412) / 9, abs=0.5)  # whole ns
    # reads: FETCH_SIZE (1000 B per timed dispatch) over the copy's scale 0.5; writes:
    # WRITE_SIZE (2048 B) over the copy's scale 1; the request sizes cross-check the reads
    # (32 + 2 * 64 + 3 * 128 bytes per timed dispatch)
    assert float(kv["fetch_scale"]) == pytest.approx(0.5) and float(kv["write_scale"]) == pytest.approx(1.0)
    assert float(kv["read_bytes_per_dispatch"]) == pytest.approx(2000)
    assert float(kv["write_bytes_per_dispatch"]) == pytest.approx(2048)
    assert float(kv["hbm_bytes_per_dispatch"]) == pytest.approx(2000 + 2048)
    assert float(kv["read_bytes_from_request_sizes"]) == pytest.approx(32 + 128 + 384)
    kp = bench._kv(str(out / "pbas_step_1280x720_n35.txt"))
    assert float(kp["avg_duration_ns"]) == pytest.approx(200)
    text = (out / "pbas_step_1280x720_n35.txt").read_text()
    assert "(1.0000 x the copy's bytes read)" in text and "FETCH_SIZE 0.5000" in text
    # bench reads the traffic back while the sources' hash matches, and not after a change
    assert bench.measured_traffic("pbas_step_1280x720_n35.txt") == pytest.approx(2000 + 2048)
    # per model-frame: a PBAS dispatch of the benchmark steps 4 models, a GMM one 8
    assert bench.measured_traffic_per_model("pbas_step_1280x720_n35.txt") == pytest.approx((2000 + 2048) / 4)
    assert bench.measured_traffic_per_model("gmm_step_1280x720_k5.txt") == pytest.approx((2000 + 2048) / 8)
    src = os.path.join(bench.ROOT, bench.STEP_KERNELS["pbas_step_1280x720_n35.txt"][2][0])
    with open(src, "a") as fh:
        fh.write(" changed")
    assert bench.measured_traffic("pbas_step_1280x720_n35.txt") is None
    table = (out / "bench_1280x720_kernel_stats.md").read_text()
    assert "| gmm_step_kernel<8, 5, 5, true, false, 1> | 9 |" in table
