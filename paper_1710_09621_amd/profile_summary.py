"""Summaries of rocprofv3 output for profiles/ (run on the host after a profiled run).

    python -m paper_1710_09621_amd.profile_summary trace  DIR BENCH_JSON OUT_MD  "COMMAND"
    python -m paper_1710_09621_amd.profile_summary traffic FETCH_DIR WRITE_DIR OUT_JSON "FETCH_COMMAND" "WRITE_COMMAND" \
        [FETCH_STDOUT]
    python -m paper_1710_09621_amd.profile_summary hmc DIR RUN1.jsonl,RUN2.jsonl OUT_MD "TRACE_COMMAND" "RUN_COMMAND"
    python -m paper_1710_09621_amd.profile_summary hmc_eq RUN.jsonl OUT_MD "RUN_COMMAND"
    python -m paper_1710_09621_amd.profile_summary hmc_compare RUN.jsonl OUT_MD "RUN_COMMAND" [paper]
    python -m paper_1710_09621_amd.profile_summary force DIR OUT_MD "COMMAND"
    python -m paper_1710_09621_amd.profile_summary cg_traffic FETCH_DIR WRITE_DIR FETCH_STDOUT OUT_MD "FETCH_COMMAND" \
        "WRITE_COMMAND"

trace: the per-kernel table of a `rocprofv3 --kernel-trace --stats` run of bench.py and, for the benchmark's
dominant kernel (the FP64 hop K1 of the schedule the bench picked), the average duration of its launches in
the timed steps next to the bench's own HIP-event figure.

traffic: HBM bytes per launch of the FP64 hop under each profiled schedule from two `rocprofv3 --pmc` passes
of profile_hop.py (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads
for k_site, which reads and writes exactly one FP64 half field; the result carries a hash of the kernel
sources so that bench.py drops it once the kernels change.  The schedules, in launch order, come from the
JSON lines profile_hop.py printed in the FETCH_SIZE run (FETCH_STDOUT), else from the --sched options of
FETCH_COMMAND.

cg_traffic: the same two counters for the five kernels of one FP64 CG iteration (profile_hop.py --cg N: the last N
launches of each), scaled by the same k_site calibration, against the algorithmic bytes the library's kernel
timing reports for each kernel (from the JSON line of the FETCH_SIZE run).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1710_09621_amd/csrc/kernels.hip", "paper_1710_09621_amd/csrc/eofa_dev.h",
                  "paper_1710_09621_amd/csrc/eofa_int.h"]


def _rows(pattern):
    out = []
    for path in sorted(glob.glob(pattern, recursive=True)):
        with open(path, newline="") as f:
            out += list(csv.DictReader(f))
    return out


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(f"none of {names} in {list(row)}")


def source_sha1():
    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def hop_kernel_name(sched):
    """Kernel-name prefix of the FP64 K1 hop (u = A_T^{-1} H_eo p, HM_SITE = 1) under schedule sched."""
    if sched[0] == 6:
        return "eofa::k_hop_tws<16, false, 1, false, double>"
    if sched[0] == 5:
        return "eofa::k_hop_tw<16, false, 1, false, double, true>"
    if sched[0] == 3:
        return "eofa::k_hop_tw<16, false, 1, false, double, false>"
    return "eofa::k_hop<16, false, 1, false, double>"


def trace(d, bench_json, out_md, command):
    stats = _rows(os.path.join(d, "**", "*kernel_stats.csv"))
    kt = _rows(os.path.join(d, "**", "*kernel_trace.csv"))
    with open(bench_json) as f:
        b = json.loads([ln for ln in f if ln.startswith("{")][-1])
    sched = b["schedules"]["fp64"]
    name = hop_kernel_name(sched)
    total = sum(float(_col(r, "TotalDurationNs")) for r in stats)
    stats.sort(key=lambda r: -float(_col(r, "TotalDurationNs")))
    lines = [f"# FP64 CG iteration kernels on {b['config']['lattice']}, Ns = {b['config']['Ns']}: bench kernel trace", "",
             "Command (repository root, GPU box):", "", f"    {command}", "",
             f"The run: autotune of the hop schedules, {b['warmup']} warm-up and {b['steps']} timed steps; one step = "
             f"{b['config']['workload'].split('; one step = ')[-1]}.", "",
             "## Top kernels (rocprofv3 --stats, whole run)", "", "| kernel | calls | avg us | total % |",
             "|---|---:|---:|---:|"]
    for r in stats[:14]:
        nm = _col(r, "Name", "KernelName", "Kernel_Name").replace("|", "\\|")
        lines.append(f"| `{nm[:110]}` | {_col(r, 'Calls')} | {float(_col(r, 'AverageNs')) / 1e3:.1f} | "
                     f"{100 * float(_col(r, 'TotalDurationNs')) / total:.2f} |")
    # launches of the dominant kernel in time order; the last steps * niter are the timed steps' K1 launches
    k1 = [r for r in kt if _col(r, "Kernel_Name", "KernelName", "Name").replace("void ", "").startswith(name)]
    k1.sort(key=lambda r: int(_col(r, "Start_Timestamp")))
    n_timed = b["steps"] * b["config"]["cg_iterations_per_step"]
    dur = [(int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3 for r in k1]
    timed = dur[-n_timed:]
    avg = sum(timed) / len(timed)
    alg = b["roofline"]["alg_bytes_per_launch"]
    lines += ["", f"## Dominant kernel `{name}` (FP64 schedule {sched} picked by the autotuner)", "",
              f"- launches in the run: {len(dur)} (autotune candidates and warm-up included)",
              f"- launches in the timed steps: {n_timed}; their average duration in the trace: **{avg:.1f} us**",
              f"- bench.py in the same run (HIP events around each launch): {b['roofline']['avg_launch_ms'] * 1e3:.1f} us, "
              f"{b['value']:.0f} GB/s algorithmic ({alg / 1e9:.3f} GB per launch), frac {b['roofline']['frac']:.3f} of 8 TB/s",
              f"- from the trace average: {alg / (avg * 1e-6) / 1e9:.0f} GB/s, frac {alg / (avg * 1e-6) / 8e12:.3f}", "",
              "## One FP64 CG iteration (bench.py, HIP events)", "",
              "| kernel | ms per launch | GB/s algorithmic |", "|---|---:|---:|"]
    for k, v in b["cg_iteration"]["kernels"].items():
        lines.append(f"| {k} | {v['ms']:.4f} | {v['gbs']:.0f} |")
    it = b["cg_iteration"]
    lines += [f"| whole iteration | {it['ms']:.3f} | {it['gbs']:.0f} (frac {it['frac']:.3f}) |", ""]
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    print(out_md, f"K1 trace avg {avg:.1f} us vs bench {b['roofline']['avg_launch_ms'] * 1e3:.1f} us")


def _per_dispatch(d, counter):
    """[(kernel name, value)] per dispatch in dispatch order."""
    rows = _rows(os.path.join(d, "**", "*counter_collection.csv"))
    out = {}
    for r in rows:
        if _col(r, "Counter_Name") != counter:
            continue
        did = int(_col(r, "Dispatch_Id"))
        nm = _col(r, "Kernel_Name")
        out.setdefault(did, [nm, 0.0])[1] += float(_col(r, "Counter_Value"))
    return [tuple(out[k]) for k in sorted(out)]


def traffic(fetch_dir, write_dir, out_json, fetch_cmd, write_cmd, fetch_stdout=None, dims=(32, 32, 32, 64), Ns=16,
            nrep=3):
    import re
    if fetch_stdout:
        with open(fetch_stdout) as fo:
            scheds = [",".join(map(str, json.loads(ln)["schedule"])) for ln in fo if ln.startswith("{")]
    else:
        scheds = [s.split()[0] for s in re.findall(r"--sched (\S+)", fetch_cmd)]
    f = _per_dispatch(fetch_dir, "FETCH_SIZE")
    w = _per_dispatch(write_dir, "WRITE_SIZE")
    Vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    half = Vh * 12 * Ns * 16
    cal_f = [v for nm, v in f if "k_site<16, false, double>" in nm]
    cal_w = [v for nm, v in w if "k_site<16, false, double>" in nm]
    ff = half / (sum(cal_f) / len(cal_f) * 1024)
    wf = half / (sum(cal_w) / len(cal_w) * 1024)
    alg = Vh * (2 * 12 * Ns * 16 + 8 * 9 * 16)
    res = {"kernel": "FP64 fused hop with the A_T^-1 epilogue (k_hop / k_hop_tw / k_hop_tws <16, false, HM_SITE, false, double>)",
           "lattice": "x".join(map(str, dims)), "Ns": Ns, "commands": [fetch_cmd, write_cmd],
           "calibration": {"kernel": f"k_site<16, false, double> (reads and writes one FP64 half field, {half} bytes "
                                     "each way)", "fetch_kib": cal_f, "write_kib": cal_w,
                           "fetch_factor": round(ff, 4), "write_factor": round(wf, 4)},
           "kernels": "schedule mode 0/1: k_hop, 3: k_hop_tw, 5: k_hop_tw with the x neighbours from LDS, 6: k_hop_tws",
           "algorithmic_bytes_per_launch": alg, "by_schedule": {}, "source_sha1": source_sha1(),
           "source_files": KERNEL_SOURCES}

    def hops(rows):
        return [v for nm, v in rows if re.search(r"k_hop(_tws?)?<16, false, 1, false, double", nm)]
    hf, hw = hops(f), hops(w)
    assert len(hf) == len(hw) == len(scheds) * (nrep + 2), (len(hf), len(hw), len(scheds))
    # profile_hop.py: per schedule, 2 untimed + nrep timed launches; keep the nrep timed ones
    per = nrep + 2
    for i, s in enumerate(scheds):
        fk = hf[i * per + 2:(i + 1) * per]
        wk = hw[i * per + 2:(i + 1) * per]
        rd = ff * 1024 * sum(fk) / len(fk)
        wr = wf * 1024 * sum(wk) / len(wk)
        # one row per candidate of the autotuner (fields as in by_schedule_fields)
        res["by_schedule"][s] = [round(rd), round(wr), round(rd + wr), round((rd + wr) / alg, 4)]
    res["by_schedule_fields"] = ["read_bytes_per_launch", "write_bytes_per_launch", "bytes_per_launch",
                                 "amplification"]
    rows = res.pop("by_schedule")
    text = json.dumps(res, indent=1)[:-2]
    text += ',\n "by_schedule": {\n' + ",\n".join(f'  "{k}": {json.dumps(v)}' for k, v in rows.items()) + "\n }\n}\n"
    json.loads(text)
    with open(out_json, "w") as fo:
        fo.write(text)
    res["by_schedule"] = {k: {"amplification": v[3]} for k, v in rows.items()}
    print(out_json, {k: v["amplification"] for k, v in res["by_schedule"].items()})


CG_KERNELS = [("hop", "K1 u = A_T^-1 H_eo p"), ("schur_w", "K2 w = Dhat p, wt = A_T^-dag w, ‖w‖²"),
              ("hop_dag", "K3 at = A_T^-dag g5 H_eo g5 wt"), ("schur_q", "K4 r -= alpha (w - H_oe at / 4), ‖r‖²"),
              ("xp", "K5 x += alpha p, p = r + beta p")]


def _cg_class(name):
    """K1..K5 key of a kernel name of the FP64 CG iteration, else None."""
    import re
    if "k_cg_xp<double" in name:
        return "xp"
    m = re.search(r"k_hop(?:_tws?)?<16, (false|true), (\d), (?:false|true), double", name)
    if not m:
        return None
    return {("false", "1"): "hop", ("false", "2"): "schur_w", ("true", "1"): "hop_dag",
            ("true", "3"): "schur_q"}.get((m.group(1), m.group(2)))


def cg_traffic(fetch_dir, write_dir, fetch_stdout, out_md, fetch_cmd, write_cmd):
    with open(fetch_stdout) as fo:
        info = [json.loads(ln) for ln in fo if ln.startswith("{") and "cg_iters" in ln][-1]
    dims, Ns, n = tuple(info["dims"]), info["Ns"], info["cg_iters"]
    f = _per_dispatch(fetch_dir, "FETCH_SIZE")
    w = _per_dispatch(write_dir, "WRITE_SIZE")
    Vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    half = Vh * 12 * Ns * 16
    cal_f = [v for nm, v in f if "k_site<16, false, double>" in nm]
    cal_w = [v for nm, v in w if "k_site<16, false, double>" in nm]
    ff = half / (sum(cal_f) / len(cal_f) * 1024)
    wf = half / (sum(cal_w) / len(cal_w) * 1024)
    lines = ["# FP64 CG iteration kernels on %s, Ns = %d: measured HBM traffic" % ("x".join(map(str, dims)), Ns), "",
             "Commands (repository root, GPU box; `cd /tmp && export TMPDIR=/tmp` first):", "",
             "    " + fetch_cmd, "    " + write_cmd, "",
             "Schedule %s; %d CG iterations of the benchmark step (action (+1, 0.01, 0.1, 1.0)), the last %d launches "
             "of each kernel. Counters in KiB per dispatch, scaled by what they read for `k_site<16, false, double>` "
             "(one FP64 half field of %d bytes read and one written): FETCH_SIZE x %.4f, WRITE_SIZE x %.4f "
             "(calibration dispatches: %d)." % (info["schedule"], n, n, half, ff, wf, len(cal_f)), "",
             "| kernel | algorithmic GB | read GB | written GB | measured GB | measured / algorithmic |",
             "|---|---:|---:|---:|---:|---:|"]
    tot = [0.0, 0.0, 0.0]
    for key, desc in CG_KERNELS:
        fk = [v for nm, v in f if _cg_class(nm) == key][-n:]
        wk = [v for nm, v in w if _cg_class(nm) == key][-n:]
        assert len(fk) == len(wk) == n, (key, len(fk), len(wk))
        k = info["kernels"][key]
        alg = k["bytes"] / k["launches"]
        rd = ff * 1024 * sum(fk) / n
        wr = wf * 1024 * sum(wk) / n
        tot[0] += alg
        tot[1] += rd
        tot[2] += wr
        lines.append("| %s | %.3f | %.3f | %.3f | %.3f | %.3f |" % (desc, alg / 1e9, rd / 1e9, wr / 1e9,
                                                                   (rd + wr) / 1e9, (rd + wr) / alg))
    lines.append("| one iteration | %.3f | %.3f | %.3f | %.3f | %.3f |" % (tot[0] / 1e9, tot[1] / 1e9, tot[2] / 1e9,
                                                                          (tot[1] + tot[2]) / 1e9,
                                                                          (tot[1] + tot[2]) / tot[0]))
    with open(out_md, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def hmc(d, runs, out_md, command, run_command):
    """Kernel-time split of one HMC trajectory (rocprofv3 --stats of hmc.py) and the per-trajectory lines of the
    three splittings (hmc.py --out files, comma-separated)."""
    stats = _rows(os.path.join(d, "**", "*kernel_stats.csv"))
    total = sum(float(_col(r, "TotalDurationNs")) for r in stats)
    groups = {"gauge force + kick": ("k_gauge_force",), "link update": ("k_link_update",),
              "link packing": ("k_pack_links",), "fermion force": ("k_force<",),
              "plaquette action": ("k_plaquette",)}
    split = {k: 0.0 for k in groups}
    split["solves (hops, CG updates and reductions, sources, heat-bath)"] = 0.0
    for r in stats:
        nm = _col(r, "Name", "KernelName", "Kernel_Name")
        t = float(_col(r, "TotalDurationNs"))
        for g, keys in groups.items():
            if any(k in nm for k in keys):
                split[g] += t
                break
        else:
            split["solves (hops, CG updates and reductions, sources, heat-bath)"] += t
    lines = ["# HMC trajectories of one-flavour EOFA on 16x16x16x32, Ns = 16", "",
             "Trajectories (repository root, GPU box):", "", f"    {run_command}", "",
             "| splitting | trajectory | dH | accepted | seconds | heat-bath s | MD s | CG iterations | force evaluations (k0, k1, k2) |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---|"]
    for path in runs.split(","):
        with open(path) as f:
            rows = [json.loads(ln) for ln in f if ln.strip()]
        summ = [r["summary"] for r in rows if "summary" in r][0]
        for r in rows:
            if "summary" in r:
                continue
            lines.append(f"| {summ['scheme']} ({len(summ['actions'])} actions) | {r['traj']} | {r['dH']:.3f} | "
                         f"{r['accepted']} | {r['seconds']:.2f} | {r['heatbath_s']:.2f} | {r['md_s']:.2f} | "
                         f"{r['cg_iters']} | {r['force_evals']} |")
    lines += ["", "Kernel trace of one new-MP trajectory:", "", f"    {command}", "",
              "| part | device time ms | share |", "|---|---:|---:|"]
    for g, t in sorted(split.items(), key=lambda kv: -kv[1]):
        lines.append(f"| {g} | {t / 1e6:.1f} | {100 * t / total:.1f}% |")
    stats.sort(key=lambda r: -float(_col(r, "TotalDurationNs")))
    lines += ["", "| kernel | calls | avg us | total % |", "|---|---:|---:|---:|"]
    for r in stats[:12]:
        nm = _col(r, "Name", "KernelName", "Kernel_Name").replace("|", "\\|")
        lines.append(f"| `{nm[:100]}` | {_col(r, 'Calls')} | {float(_col(r, 'AverageNs')) / 1e3:.1f} | "
                     f"{100 * float(_col(r, 'TotalDurationNs')) / total:.2f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out_md, {k: round(v / 1e6, 1) for k, v in split.items()})


def force(d, out_md, command, dims=(32, 32, 32, 64), Ns=16):
    """Kernel table of a rocprofv3 --stats run of profile_force.py and the fermion-force kernel's rate."""
    stats = _rows(os.path.join(d, "**", "*kernel_stats.csv"))
    total = sum(float(_col(r, "TotalDurationNs")) for r in stats)
    stats.sort(key=lambda r: -float(_col(r, "TotalDurationNs")))
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    lines = [f"# EOFA fermion force (k_force) on {'x'.join(map(str, dims))}, Ns = {Ns}", "",
             "Command (repository root, GPU box):", "", f"    {command}", "",
             "The driver computes the force of the new-MP middle action (+, 0.01, 0.1; 1.0) twice with the FP16-storage",
             "solver; each force call launches `k_force` once per parity.", "",
             "| kernel | calls | avg us | total % |", "|---|---:|---:|---:|"]
    for r in stats[:10]:
        nm = _col(r, "Name", "KernelName", "Kernel_Name").replace("|", "\\|")
        lines.append(f"| `{nm[:100]}` | {_col(r, 'Calls')} | {float(_col(r, 'AverageNs')) / 1e3:.1f} | "
                     f"{100 * float(_col(r, 'TotalDurationNs')) / total:.2f} |")
    kf = [r for r in stats if f"k_force<{Ns}>" in _col(r, "Name", "KernelName", "Kernel_Name")][0]
    avg = float(_col(kf, "AverageNs")) / 1e3
    # per launch (one parity's links): the 5D solution on both parities once, the links of one parity, the force out
    alg = V * Ns * 12 * 16 + (V // 2) * 4 * 144 + (V // 2) * 4 * 8 * 8
    lines += ["", f"`k_force<{Ns}>`: {_col(kf, 'Calls')} launches, average {avg:.1f} us per parity. Algorithmic bytes per "
              f"launch (one parity's links): the 5D solution on both parities once ({V * Ns * 192 / 1e9:.2f} GB), the "
              f"links of one parity ({(V // 2) * 576 / 1e9:.2f} GB) and the force of one parity "
              f"({(V // 2) * 256 / 1e9:.3f} GB) = {alg / 1e9:.2f} GB, i.e. {alg / (avg * 1e-6) / 1e12:.2f} TB/s "
              f"({100 * alg / (avg * 1e-6) / 8e12:.0f}% of 8 TB/s)."]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out_md, f"k_force {avg:.1f} us")


# The maximum fermion forces per factor and the time per trajectory that Sec. III prints for one-flavour QCD on its
# 24^3 x 48 ensembles at beta = 6.20 with m_q = 0.005, m_h = 0.1 (bare; 0.005 / 2.6 and 0.1 / 2.6 normalised)
PAPER_NF1 = {"none": dict(forces=[0.0830, 0.2529], seconds=46162, acceptance=0.97),
             "old": dict(forces=[0.0012, 0.0040, 0.0234, 0.2244], seconds=22839, acceptance=0.88),
             "new": dict(forces=[0.0011, 0.0348, 0.2243], seconds=18346, acceptance=0.88)}


def hmc_compare(run, out_md, run_command, paper=""):
    """The three splittings from one thermalised field (hmc.py --therm N --compare): per splitting the time, CG
    iterations, acceptance and the force magnitudes per action."""
    with open(run) as f:
        rows = [json.loads(ln) for ln in f if ln.strip()]
    therm = [r for r in rows if r.get("phase") == "therm"]
    summs = [r["summary"] for r in rows if "summary" in r]
    lat = summs[0]
    lines = [f"# The splittings of Sec. III from one thermalised field: {lat['lattice']}, Ns = {lat['Ns']}", "",
             "Command (repository root, GPU box):", "", f"    {run_command}", "",
             f"beta = {lat['beta']}, (k0, k1, k2) = {tuple(lat['steps'])}, {lat['prec']} solves to 1e-10 (interior force "
             f"solves to {lat.get('force_tol') or 1e-10:g}), chronological "
             f"start vectors: {lat['chrono']}. {len(therm)} thermalisation trajectories of the "
             f"{therm[0]['scheme'] if therm else '-'} splitting with (m, m_h, M) = "
             f"{tuple(therm[0].get('masses', [])) if therm else '-'} (plaquette {therm[0]['plaquette'] if therm else 0:.4f} -> "
             f"{therm[-1]['plaquette'] if therm else 0:.4f}); then every splitting runs {lat['ntraj']} trajectories from "
             "the same field. ‖F‖ = sqrt(sum_a F^a F^a) averaged over the links; per action the largest over its force "
             "evaluations in a trajectory (mean over the trajectories).", "",
             "| splitting | actions (level, chir, m3, m4, mo) | seconds per trajectory | CG iterations | accepted | largest ‖F‖ per action | gauge ‖F‖ |",
             "|---|---|---:|---:|---:|---|---:|"]
    for sm in summs:
        acts = "; ".join(f"({a[0]}, {a[1]:+d}, {a[2]}, {a[3]}, {a[4]})" for a in sm["actions"])
        lines.append(f"| {sm['scheme']} | {acts} | {sm['mean_s']:.2f} | {sm['mean_cg']:.0f} | {sm['accepted']}/{sm['ntraj']} | "
                     f"{', '.join(f'{v:.4f}' for v in sm['force_max'])} | {sm['gauge_force0']:.3f} |")
    if paper:
        lines += ["", "The same quantities as printed in Sec. III for one-flavour QCD (24³×48, β = 6.20, m_q = 0.005, "
                  "m_h = 0.1 bare, i.e. the normalised masses of this run; other hardware and volume):", "",
                  "| splitting | largest ‖F‖ per action, Sec. III | this run | seconds per trajectory, Sec. III (ratio to new MP) "
                  "| this run (ratio to new MP) |", "|---|---|---|---:|---:|"]
        ours = {sm["scheme"]: sm for sm in summs}
        for k in ("new", "old", "none"):
            if k not in ours:
                continue
            pp, o = PAPER_NF1[k], ours[k]
            lines.append(f"| {k} | {', '.join(f'{v:.4f}' for v in pp['forces'])} | "
                         f"{', '.join(f'{v:.4f}' for v in o['force_max'])} | {pp['seconds']} "
                         f"({pp['seconds'] / PAPER_NF1['new']['seconds']:.2f}) | {o['mean_s']:.1f} "
                         f"({o['mean_s'] / ours['new']['mean_s']:.2f}) |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out_md)


def hmc_eq(run, out_md, run_command):
    """Thermalisation history and equilibrium averages of a long hmc.py run (--out file)."""
    with open(run) as f:
        rows = [json.loads(ln) for ln in f if ln.strip()]
    summ = [r["summary"] for r in rows if "summary" in r][0]
    traj = [r for r in rows if "summary" not in r]
    lines = [f"# HMC equilibrium check on {summ['lattice']}, Ns = {summ['Ns']} ({summ['scheme']} MP)", "",
             "Command (repository root, GPU box):", "", f"    {run_command}", "",
             f"beta = {summ['beta']}, (k0, k1, k2) = {tuple(summ['steps'])}, actions (level, chir, m3, m4, mo) = "
             f"{summ['actions']}, {summ['prec']} solves to 1e-10, chronological start vectors: {summ.get('chrono')}.", "",
             f"Over the {summ['ntraj'] - summ['burn']} trajectories after the first {summ['burn']}:", "",
             f"- <exp(-dH)> = {summ['exp_mdH']:.4f} +- {summ['exp_mdH_err']:.4f} (1 in equilibrium for a reversible, "
             "area-preserving integrator)",
             f"- acceptance {summ['acceptance']:.3f}, mean |dH| {summ['mean_abs_dH']:.4f}",
             f"- plaquette {summ['plaquette']:.4f}; mean time per trajectory {summ['mean_s']:.3f} s, "
             f"{summ['mean_cg']:.0f} CG iterations", "",
             "| trajectory | plaquette | dH | accepted | CG iterations | seconds |", "|---:|---:|---:|---:|---:|---:|"]
    for i, r in enumerate(traj):
        if i < 10 or i % 10 == 0 or i == len(traj) - 1:
            lines.append(f"| {r['traj']} | {r['plaquette']:.4f} | {r['dH']:.4f} | {r['accepted']} | {r['cg_iters']} | "
                         f"{r['seconds']:.3f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out_md)


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(*sys.argv[2:6])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:8])
    elif sys.argv[1] == "hmc":
        hmc(*sys.argv[2:7])
    elif sys.argv[1] == "force":
        force(*sys.argv[2:5])
    elif sys.argv[1] == "hmc_compare":
        hmc_compare(*sys.argv[2:6])
    elif sys.argv[1] == "hmc_eq":
        hmc_eq(*sys.argv[2:5])
    elif sys.argv[1] == "cg_traffic":
        cg_traffic(*sys.argv[2:8])
    else:
        raise SystemExit(__doc__)
