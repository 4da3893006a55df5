"""Host logic of the benchmark: the rocprofv3 summaries it commits and the
traffic record it reports only while the step-kernel sources match it.
Synthetic profiler outputs, no GPU."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import workloads as W  # noqa: E402

STEP0 = "void fnlb::(anonymous namespace)::k_step<float, float, 0, false>(fnlb::StepArgs)"
STEP1 = "void fnlb::(anonymous namespace)::k_step<float, float, 1, false>(fnlb::StepArgs)"
COPY = "__amd_rocclr_copyBuffer"


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


@pytest.fixture
def profiler_dirs(tmp_path):
    pt, pf, pw = (tmp_path / d for d in ("pt", "pf", "pw"))
    for d in (pt, pf, pw):
        d.mkdir()
    _write_csv(pt / "run_kernel_stats.csv", [
        dict(Name=STEP0, Calls=5, AverageNs=1000.0, Percentage=80.0),
        dict(Name=STEP1, Calls=1, AverageNs=2000.0, Percentage=20.0)])

    def launch(name, start, dur, grid):
        return dict(Kernel_Name=name, Start_Timestamp=start, End_Timestamp=start + dur,
                    Grid_Size_X=grid)
    # the roofline leg first: its clock-ramp and probe launches (excluded), two
    # timed plain launches at the timed grid (averaged), one at another grid;
    # then the sampled run: a sampling step and plain steps after it (excluded)
    lead = [launch(STEP0, 10 + k, 5000, 1024) for k in range(bench.ROOFLINE_LEAD_STEPS)]
    _write_csv(pt / "run_kernel_trace.csv", (lead + [
        launch(STEP0, 300, 1000, 1024), launch(STEP0, 400, 3000, 1024),
        launch(STEP0, 500, 7000, 2048), launch(STEP1, 600, 9000, 1024),
        launch(STEP0, 700, 5000, 1024), launch(STEP0, 800, 1000, 2048)])[::-1])

    def counter(name, kernel, value, grid=0):
        return dict(Kernel_Name=kernel, Counter_Name=name, Counter_Value=value, Grid_Size=grid)
    # the plain 1 GiB copies read half the counter's nominal bytes (so FETCH is
    # scaled x2) and write all of them (x1); a small copy is ignored
    _write_csv(pf / "run_counter_collection.csv", [
        counter("FETCH_SIZE", COPY, 524288.0), counter("FETCH_SIZE", COPY, 524288.0),
        counter("FETCH_SIZE", COPY, 10.0), counter("FETCH_SIZE", STEP0, 100.0, 1024),
        counter("FETCH_SIZE", STEP0, 300.0, 1024), counter("FETCH_SIZE", STEP0, 9999.0, 2048)])
    _write_csv(pw / "run_counter_collection.csv", [
        counter("WRITE_SIZE", COPY, 1048576.0), counter("WRITE_SIZE", STEP0, 50.0, 1024)])
    return pt, pf, pw


def test_summarize_profile_scales_counters_and_picks_the_roofline_leg(
        profiler_dirs, tmp_path, monkeypatch):
    traffic = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(traffic))
    pt, pf, pw = profiler_dirs
    md = tmp_path / "summary.md"
    bench.summarize_profile(str(pt), str(pf), str(pw), str(md), "the commands")
    d = json.loads(traffic.read_text())
    assert d["grid"] == 1024
    assert d["step_avg_us"] == pytest.approx(2.0)  # (1000 + 3000) ns / 2
    assert d["read_bytes"] == round(200.0 * 2 * 1024)  # mean FETCH x2, in bytes
    assert d["write_bytes"] == round(50.0 * 1024)
    assert d["bytes_per_launch"] == d["read_bytes"] + d["write_bytes"]
    assert d["algorithmic_bytes"] == 144 * sum(r.Lx * r.Lz for r in W.batched_ensemble(96))
    assert d["source_sha256"] == bench._step_source_hash("k_step")
    assert d["kernel"] == "k_step" and d["steps_per_launch"] == 1
    text = md.read_text()
    assert "the commands" in text and "FETCH x2.0000, WRITE x1.0000" in text
    # the record is reported for its kernel while the kernel sources match it,
    # and not after
    assert bench._traffic_from_profiles("k_step") == d["bytes_per_launch"]
    assert bench._traffic_from_profiles("k_step2") is None
    d["source_sha256"] = "0" * 64
    traffic.write_text(json.dumps(d))
    assert bench._traffic_from_profiles("k_step") is None
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "missing.json"))
    assert bench._traffic_from_profiles("k_step") is None


def test_summarize_profile_of_the_two_step_kernel(tmp_path, monkeypatch):
    """A run of the two-step kernel: its launches are the step kernel, and the
    algorithmic bytes of a launch count its two steps."""
    traffic = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(traffic))
    pt, pf, pw = (tmp_path / d for d in ("pt", "pf", "pw"))
    for d in (pt, pf, pw):
        d.mkdir()
    plain = "void fnlb::(anonymous namespace)::k_step2<0>(fnlb::Step2Args)"
    sampled = "void fnlb::(anonymous namespace)::k_step2<1>(fnlb::Step2Args)"
    _write_csv(pt / "run_kernel_stats.csv", [
        dict(Name=plain, Calls=3, AverageNs=2000.0, Percentage=90.0)])
    # the roofline leg's lead launches (half as many as its lead steps), two
    # timed launches, then a sampling launch and a plain one after it
    lead = [dict(Kernel_Name=plain, Start_Timestamp=k, End_Timestamp=k + 9000, Grid_Size_X=512)
            for k in range(bench.ROOFLINE_LEAD_STEPS // 2)]
    _write_csv(pt / "run_kernel_trace.csv", lead + [
        dict(Kernel_Name=plain, Start_Timestamp=6000, End_Timestamp=8000, Grid_Size_X=512),
        dict(Kernel_Name=plain, Start_Timestamp=9000, End_Timestamp=13000, Grid_Size_X=512),
        dict(Kernel_Name=sampled, Start_Timestamp=14000, End_Timestamp=19000, Grid_Size_X=512),
        dict(Kernel_Name=plain, Start_Timestamp=20000, End_Timestamp=29000, Grid_Size_X=512)])
    _write_csv(pf / "run_counter_collection.csv", [
        dict(Kernel_Name=COPY, Counter_Name="FETCH_SIZE", Counter_Value=524288.0, Grid_Size=0),
        dict(Kernel_Name=plain, Counter_Name="FETCH_SIZE", Counter_Value=10.0, Grid_Size=512)])
    _write_csv(pw / "run_counter_collection.csv", [
        dict(Kernel_Name=COPY, Counter_Name="WRITE_SIZE", Counter_Value=1048576.0, Grid_Size=0),
        dict(Kernel_Name=plain, Counter_Name="WRITE_SIZE", Counter_Value=20.0, Grid_Size=512)])
    bench.summarize_profile(str(pt), str(pf), str(pw), str(tmp_path / "s.md"), "cmd")
    d = json.loads(traffic.read_text())
    assert d["kernel"] == "k_step2" and d["steps_per_launch"] == 2
    assert d["step_avg_us"] == pytest.approx(3.0)
    assert d["algorithmic_bytes"] == 2 * 144 * sum(r.Lx * r.Lz for r in W.batched_ensemble(96))
    assert bench._traffic_from_profiles("k_step2") == d["bytes_per_launch"]
    # the record is hashed over the two-step kernel's own sources only: an
    # edit of the one-step kernel leaves it current
    assert "k_step.hip" not in bench.STEP_SOURCES["k_step2"]
    assert d["source_sha256"] == bench._step_source_hash("k_step2") \
        != bench._step_source_hash("k_step")


def test_summarize_trace_writes_the_command_and_table(profiler_dirs, tmp_path):
    pt, _, _ = profiler_dirs
    md = tmp_path / "trace.md"
    bench.summarize_trace(str(pt), str(md), "A title", "cmd line 1\ncmd line 2")
    text = md.read_text().splitlines()
    assert text[0] == "# A title"
    assert "cmd line 1" in text and "cmd line 2" in text
    assert any(line.startswith(f"| {STEP0[:90]} | 5 | 1.0 | 80.00 |") for line in text)


def test_summarize_timeline_accounts_for_a_sample(tmp_path):
    """Synthetic graph replay: plain launches of 100 us, a sampling launch of
    120 us with 6 us idle before and 5 after it, a row pass that stretches
    the plain launch beside it to 107 us, and one column pass that stretches
    two plain launches to 150 us each for two samples."""
    S2 = "void fnlb::(anonymous namespace)::k_step2<1>(fnlb::Step2Args)"
    P2 = "void fnlb::(anonymous namespace)::k_step2<0>(fnlb::Step2Args)"
    R2 = "void fnlb::(anonymous namespace)::k_row_fft<float>(fnlb::RepInfo const*)"
    C2 = "void fnlb::(anonymous namespace)::k_col_fft<float2>(fnlb::RepInfo const*)"
    A2 = "fnlb::(anonymous namespace)::k_advance_time(long*, long)"
    rows, t = [], 0.0

    def k(name, q, start, dur):
        rows.append(dict(Kernel_Name=name, Queue_Id=q, Start_Timestamp=int(start * 1e3),
                         End_Timestamp=int((start + dur) * 1e3)))
        return start + dur

    for rep in range(2):          # two replays of a two-period graph
        for per in range(2):
            t = k(S2, 1, t + (6.0 if per else 3.0), 120.0)
            t += 5.0
            k(R2, 3, t + 1.0, 40.0)   # beside the next plain launch
            t = k(P2, 1, t, 107.0)
            if per == 1:
                k(C2, 3, t + 1.0, 200.0)
                t = k(P2, 1, t, 150.0)
                t = k(P2, 1, t, 150.0)
            else:
                t = k(P2, 1, t, 100.0)
                t = k(P2, 1, t, 100.0)
            t = k(P2, 1, t, 100.0)
        t = k(A2, 1, t, 2.0)
    d = tmp_path / "tl"
    d.mkdir()
    _write_csv(d / "run_kernel_trace.csv", rows)
    r = bench.summarize_timeline(str(d), str(tmp_path / "tl.md"), "T", "cmd")
    assert r["plain"] == pytest.approx(100.0)
    assert r["sampling_extra"] == pytest.approx(20.0)
    assert r["gap_before"] == pytest.approx(6.0)   # the first node of a replay is left out
    assert r["gap_after"] == pytest.approx(5.0)
    assert r["beside_row"] == pytest.approx(7.0)
    assert r["col_per_sample"] == pytest.approx(4 * 50.0 / 4)
    assert r["per_sample"] == pytest.approx(20 + 6 + 5 + 7 + 50)
    # the periods without a column pass: 6 + 120 + 5 + 107 + 100 + 100 + 100 over 5 plain
    assert r["period_extra"] == pytest.approx(6 + 20 + 5 + 7)
    assert "cmd" in (tmp_path / "tl.md").read_text()


def test_more_than_one_gpu_is_refused():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
