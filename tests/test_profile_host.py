"""Host logic of the measurement, on synthetic counter files: the kernel classes and the byte scaling of the
rocprofv3 summaries (profile_summary.py) and the benchmark's use of a committed counter summary (bench.py), which
must drop the figure when the kernel sources, the lattice or the schedule do not match."""
import csv
import json
import os

import pytest

import bench
from paper_1710_09621_amd import profile_summary as PS

# kernel names as the trace prints them (arguments shortened)
K = {
    "hop": "void eofa::k_hop_tws<16, false, 1, false, double>(eofa::HopArgs<double>)",
    "hop_tw": "void eofa::k_hop_tw<16, false, 1, false, double, true>(eofa::HopArgs<double>)",
    "hop_tiled": "void eofa::k_hop<16, false, 1, false, double>(eofa::HopArgs<double>)",
    "schur_w": "void eofa::k_hop_tws<16, false, 2, true, double>(eofa::HopArgs<double>)",
    "hop_dag": "void eofa::k_hop_tws<16, true, 1, false, double>(eofa::HopArgs<double>)",
    "schur_q": "void eofa::k_hop_tws<16, true, 3, true, double>(eofa::HopArgs<double>)",
    "xp": "void eofa::k_cg_xp<double, true>(eofa::cpx<double>*, eofa::cpx<double>*, double const*, unsigned long)",
    "xp_cached": "void eofa::k_cg_xp<double, false>(eofa::cpx<double>*, eofa::cpx<double>*, double const*, unsigned long)",
    "site": "void eofa::k_site<16, false, double>(eofa::cpx<double> const*, eofa::cpx<double>*, eofa::SiteOp const*, int)",
    "mr": "void eofa::k_hop_mr<16, false, 2, float, true>(eofa::HopArgsMR<float>)",
    "xp_mr": "void eofa::k_cg_xp_mr<double, true>(eofa::XpArgs<double>, double*, unsigned long)",
    "fp32": "void eofa::k_hop_tws<16, false, 1, false, float>(eofa::HopArgs<float>)",
    "dt": "void eofa::k_hop_tws<16, false, 4, false, double>(eofa::HopArgs<double>)",
}


def test_cg_kernel_classes():
    want = {"hop": "hop", "hop_tw": "hop", "hop_tiled": "hop", "schur_w": "schur_w", "hop_dag": "hop_dag",
            "schur_q": "schur_q", "xp": "xp", "xp_cached": "xp", "site": None, "mr": None, "xp_mr": None,
            "fp32": None, "dt": None}
    for k, cls in want.items():
        assert PS._cg_class(K[k]) == cls, k


def _counters(d, counter, dispatches):
    """A counter_collection.csv with one row per (kernel name, KiB); a value given as a pair is split over two
    rows of the same dispatch (the summaries add them)."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (nm, v) in enumerate(dispatches):
            for part in (v if isinstance(v, tuple) else (v,)):
                w.writerow([i + 1, nm, counter, part])
                w.writerow([i + 1, nm, "OTHER_COUNTER", 1e9])  # other counters of the pass are ignored


DIMS, NS = (4, 4, 4, 4), 16
VH = 4 * 4 * 4 * 4 // 2
HALF = VH * 12 * NS * 16  # bytes of one FP64 half field


def test_cg_traffic_scaling(tmp_path):
    """Counters are scaled by what they read for k_site (one half field in, one out); each kernel keeps its last n
    launches; the ratio is measured over the library's own algorithmic bytes."""
    n = 2
    # FETCH_SIZE counts half the bytes on this part, WRITE_SIZE all of them: calibration factors 2 and 1
    cal_f, cal_w = HALF / 2 / 1024, HALF / 1024
    fetch = {"hop": 300.0, "schur_w": 500.0, "hop_dag": 310.0, "schur_q": 600.0, "xp": 480.0}
    write = {"hop": 96.0, "schur_w": 192.0, "hop_dag": 96.0, "schur_q": 96.0, "xp": 192.0}
    names = {"hop": K["hop"], "schur_w": K["schur_w"], "hop_dag": K["hop_dag"], "schur_q": K["schur_q"],
             "xp": K["xp"]}
    # an earlier hop launch (the dslash launches before the CG) must not be counted
    fd = [(K["hop"], 1e6), (K["site"], (cal_f / 2, cal_f / 2)), (K["site"], cal_f)]
    wd = [(K["hop"], 1e6), (K["site"], cal_w), (K["site"], cal_w)]
    for _ in range(n):
        for key in ("hop", "schur_w", "hop_dag", "schur_q", "xp"):
            fd.append((names[key], fetch[key]))
            wd.append((names[key], write[key]))
    _counters(str(tmp_path / "f"), "FETCH_SIZE", fd)
    _counters(str(tmp_path / "w"), "WRITE_SIZE", wd)
    alg = {"hop": 1e6, "schur_w": 2e6, "hop_dag": 1e6, "schur_q": 2e6, "xp": 3e6}
    out = tmp_path / "stdout"
    out.write_text("setup line\n" + json.dumps(dict(dims=DIMS, Ns=NS, schedule=[6, 1, 4, 4, 64, 32, 0], cg_iters=n,
                                                     kernels={k: dict(launches=n, bytes=n * v) for k, v in alg.items()}))
                   + "\n")
    md = tmp_path / "t.md"
    PS.cg_traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(out), str(md), "FETCH cmd", "WRITE cmd")
    rows = [ln for ln in md.read_text().splitlines() if ln.startswith("| K") or ln.startswith("| one")]
    assert len(rows) == 6
    tot = 0.0
    for ln, key in zip(rows, ("hop", "schur_w", "hop_dag", "schur_q", "xp")):
        cells = [c.strip() for c in ln.strip("|").split("|")]
        rd, wr = 2 * 1024 * fetch[key], 1024 * write[key]
        assert float(cells[1]) == pytest.approx(alg[key] / 1e9, abs=5e-4)
        assert float(cells[2]) == pytest.approx(rd / 1e9, abs=5e-4)
        assert float(cells[3]) == pytest.approx(wr / 1e9, abs=5e-4)
        assert float(cells[5]) == pytest.approx((rd + wr) / alg[key], abs=5e-4)
        tot += rd + wr
    last = [c.strip() for c in rows[-1].strip("|").split("|")]
    assert float(last[5]) == pytest.approx(tot / sum(alg.values()), abs=5e-4)


def _hop_summary(tmp_path, nrep=3):
    """Counter summary of the FP64 hop under two schedules, as written by `profile_summary traffic`."""
    scheds = [[6, 1, 4, 4, 64, 32, 0], [1, 1, 4, 4, 8, 32, 0]]
    kib = {0: (2000.0, 600.0), 1: (2500.0, 610.0)}
    fd, wd = [], []
    for i, sc in enumerate(scheds):
        name = K["hop"] if sc[0] == 6 else K["hop_tiled"]
        for k in range(nrep + 2):  # 2 untimed launches first, with other values that must be skipped
            f, w = kib[i] if k >= 2 else (1e7, 1e7)
            fd.append((name, f))
            wd.append((name, w))
    fd += [(K["site"], HALF / 2 / 1024)]
    wd += [(K["site"], HALF / 1024)]
    _counters(str(tmp_path / "hf"), "FETCH_SIZE", fd)
    _counters(str(tmp_path / "hw"), "WRITE_SIZE", wd)
    out = tmp_path / "hstdout"
    out.write_text("".join(json.dumps(dict(schedule=sc)) + "\n" for sc in scheds))
    js = tmp_path / "hop_traffic.json"
    PS.traffic(str(tmp_path / "hf"), str(tmp_path / "hw"), str(js), "F", "W", str(out), dims=DIMS, Ns=NS, nrep=nrep)
    return js, scheds, kib


def test_hop_traffic_summary(tmp_path):
    js, scheds, kib = _hop_summary(tmp_path)
    t = json.loads(js.read_text())
    alg = VH * (2 * 12 * NS * 16 + 8 * 9 * 16)
    assert t["algorithmic_bytes_per_launch"] == alg and t["source_sha1"] == PS.source_sha1()
    assert t["calibration"]["fetch_factor"] == pytest.approx(2.0) and t["calibration"]["write_factor"] == 1.0
    for i, sc in enumerate(scheds):
        rd, wr, tot, amp = t["by_schedule"][",".join(map(str, sc))]
        assert rd == round(2 * 1024 * kib[i][0]) and wr == round(1024 * kib[i][1]) and tot == rd + wr
        assert amp == pytest.approx(tot / alg, abs=1e-4)


def test_bench_uses_summary_only_when_it_matches(tmp_path):
    js, scheds, kib = _hop_summary(tmp_path)
    t = json.loads(js.read_text())
    sc = scheds[0]
    got = bench.measured_traffic(str(js), DIMS, NS, sc)
    assert got == t["by_schedule"][",".join(map(str, sc))][2]
    assert bench.measured_traffic(str(js), DIMS, NS, [6, 1, 2, 4, 64, 32, 0]) is None  # schedule not profiled
    assert bench.measured_traffic(str(js), (8, 4, 4, 4), NS, sc) is None  # other lattice
    assert bench.measured_traffic(str(js), DIMS, 8, sc) is None  # other Ns
    assert bench.measured_traffic(str(tmp_path / "missing.json"), DIMS, NS, sc) is None
    t["source_sha1"] = "0" * 40  # the kernels changed since the counters were taken
    js.write_text(json.dumps(t))
    assert bench.measured_traffic(str(js), DIMS, NS, sc) is None


def test_committed_summary_matches_the_sources():
    """The committed hop counter summary was taken on the kernel sources in the tree, at the benchmark's lattice,
    and covers every schedule the autotuner can pick there."""
    path = os.path.join(PS.ROOT, "profiles", "hop_traffic.json")
    t = json.load(open(path))
    assert t["lattice"] == "32x32x32x64" and t["Ns"] == 16
    assert len(t["by_schedule"]) == 384
    assert t["by_schedule_fields"] == ["read_bytes_per_launch", "write_bytes_per_launch", "bytes_per_launch",
                                       "amplification"]
    if t["source_sha1"] != PS.source_sha1():
        # the benchmark then reports traffic = null until the two --pmc passes are taken again
        pytest.skip("kernel sources changed since profiles/hop_traffic.json was taken")
    assert bench.measured_traffic(path, (32, 32, 32, 64), 16, [6, 1, 4, 4, 64, 32, 0]) is not None
