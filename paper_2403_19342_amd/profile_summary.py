"""Summaries of rocprofv3 CSV output (kernel statistics and counters).

    python -m paper_2403_19342_amd.profile_summary stats <kernel_stats.csv>
    python -m paper_2403_19342_amd.profile_summary pmc <counter_collection.csv> COUNTER [COPY_BYTES]
    python -m paper_2403_19342_amd.profile_summary traffic <fetch.csv> <write.csv> COPY_BYTES
    python -m paper_2403_19342_amd.profile_summary trace <kernel_trace.csv>

`trace` also averages each kernel over its full launches only (duration at
least a quarter of the median): solve kernels launched past convergence in
the last group of CG iterations return at once and pull the plain mean down.

`stats` prints calls, average and total time per kernel.  `pmc` prints the
average value of COUNTER per dispatch for every kernel; with COPY_BYTES (the
bytes one plain device-to-device copy moves per direction) it also prints the
ratio counter/actual measured on the runtime's copy kernel, the factor that
turns the counter of any other kernel into bytes.
"""
from __future__ import annotations

import csv
import sys
from collections import defaultdict


def _short(name: str, width: int = 70) -> str:
    name = name.split("(")[0]
    return name if len(name) <= width else name[: width - 3] + "..."


def stats(path: str, top: int = 40) -> None:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print(f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}")
    for r in rows[:top]:
        print(f"{_short(r['Name']):70s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")


def pmc(path: str, counter: str, copy_bytes: float | None = None) -> None:
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    print(f"{'kernel':70s} {'dispatches':>10s} {'avg ' + counter + ' (KiB)':>22s}")
    for name, vals in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        print(f"{_short(name):70s} {len(vals):10d} {sum(vals) / len(vals):22.1f}")
    if copy_bytes:
        copies = [v for k, vals in acc.items() if "copyBuffer" in k for v in vals]
        big = [v for v in copies if v * 1024.0 > 0.5 * copy_bytes]
        if big:
            f = (sum(big) / len(big)) * 1024.0 / copy_bytes
            print(f"copy calibration: {len(big)} copies of {copy_bytes:.0f} B, counter/actual = {f:.4f}")


def trace(path: str, top: int = 30) -> None:
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print(f"{'kernel':70s} {'calls':>6s} {'mean_us':>9s} {'full':>6s} {'full_mean_us':>12s}")
    for name, d in sorted(acc.items(), key=lambda kv: -sum(kv[1]))[:top]:
        med = sorted(d)[len(d) // 2]
        full = [x for x in d if x >= 0.25 * med]
        print(f"{_short(name):70s} {len(d):6d} {sum(d) / len(d):9.2f} {len(full):6d} {sum(full) / len(full):12.2f}")


# kernel-name prefix -> profiling class of the solve (see specmg_get_profile)
CLASSES = {"k_spmv_pcg": "cg_spmv", "k_pre_smooth": "pre_smooth", "k_resid_restrict": "resid_restrict",
           "k_prolong": "prolong", "k_post_fused": "post_smooth", "k_p_update": "p_update",
           "k_coarsest_sym": "coarsest"}
TRAFFIC_SOURCES = ("csrc/k_fine.hip", "csrc/k_coarse.hip", "csrc/common.hpp")


def source_hash() -> str:
    """sha256 over the sources of the solve kernels whose traffic is recorded."""
    import hashlib
    import os
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(here, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _avg(path: str, counter: str) -> dict:
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            acc[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
    return acc


def _calib(acc: dict, copy_bytes: float) -> float:
    big = [v for k, vals in acc.items() if "copyBuffer" in k for v in vals if v > 0.5 * copy_bytes]
    if not big:
        raise SystemExit("no copy dispatch of the calibration size found")
    return (sum(big) / len(big)) / copy_bytes


def traffic(fetch_csv: str, write_csv: str, copy_bytes: float) -> None:
    """Per-class HBM bytes per launch: counter bytes divided by the factor the
    same counter reads on the runtime's copy kernel (copy_bytes each way)."""
    fa, wa = _avg(fetch_csv, "FETCH_SIZE"), _avg(write_csv, "WRITE_SIZE")
    ff, fw = _calib(fa, copy_bytes), _calib(wa, copy_bytes)
    print(f"calibration: FETCH_SIZE/actual = {ff:.4f}, WRITE_SIZE/actual = {fw:.4f} "
          f"(copy kernel, {copy_bytes:.0f} B each way)")
    print(f"source_sha256: {source_hash()}")
    for name in sorted(fa):
        short = name.split("(")[0].split("::")[-1].split("<")[0]
        cls = CLASSES.get(short)
        if cls is None or name not in wa:
            continue
        f = sum(fa[name]) / len(fa[name]) / ff
        w = sum(wa[name]) / len(wa[name]) / fw
        print(f"traffic {cls}: fetch_bytes={f:.0f} write_bytes={w:.0f} dispatches={len(fa[name])}")


def read_traffic(path: str) -> dict:
    """{class: bytes per launch} from a `traffic` summary, or {} when the
    fine-kernel sources changed since the counters were taken."""
    out, sha = {}, None
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return {}
    for line in lines:
        line = line.strip().strip("`")
        if line.startswith("source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("traffic "):
            cls, rest = line[len("traffic "):].split(":", 1)
            kv = dict(t.split("=") for t in rest.split())
            out[cls.strip()] = float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    return out if sha == source_hash() else {}


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        stats(argv[1])
    elif len(argv) >= 2 and argv[0] == "trace":
        trace(argv[1])
    elif len(argv) >= 4 and argv[0] == "traffic":
        traffic(argv[1], argv[2], float(argv[3]))
    elif len(argv) >= 3 and argv[0] == "pmc":
        pmc(argv[1], argv[2], float(argv[3]) if len(argv) > 3 else None)
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
