"""Summarise rocprofv3 CSV output of a benchmark run into per-kernel tables.

    python -m paper_2303_09886_amd.profsum [--traffic-json OUT] TRACE_DIR [PMC_DIR ...]

TRACE_DIR holds a ``--kernel-trace --output-format csv`` run
(``*_kernel_trace.csv``); each PMC_DIR a ``--pmc ... --output-format csv`` run
(``*_counter_collection.csv``).  Dispatches are grouped by kernel and grid
size (the benchmark runs the large and the small workload, whose dispatches
of one kernel differ in grid size); each group prints its mean duration and
the mean of every counter per dispatch.  HBM bytes are scaled with the
plain device copy of the run (the largest ``__amd_rocclr_copyBuffer``
dispatch, 512 MiB read and 512 MiB written), which reads what FETCH_SIZE and
WRITE_SIZE (KiB) mean on this GPU.

--traffic-json OUT writes, for each kernel, the HBM bytes per launch of its
largest-grid dispatches (the benchmark's large workload) with the hash of
the kernel source they were taken on; bench.py reports them as the roofline's
`traffic` while that source is unchanged.
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

COPY_BYTES = 512 << 20
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def source_hash() -> str:
    """Hash of the kernel source and its C header (first 16 hex digits)."""
    h = hashlib.sha256()
    for rel in ("paper_2303_09886_amd/csrc/fengine.hip", "include/fengine.h"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name).strip()


def load_trace(d):
    groups = collections.defaultdict(list)
    for f in glob.glob(os.path.join(d, "*_kernel_trace.csv")):
        for r in csv.DictReader(open(f)):
            grid = int(r["Grid_Size"]) if "Grid_Size" in r else \
                int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            key = (short(r["Kernel_Name"]), grid)
            groups[key].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return groups


def load_pmc(dirs):
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for f in glob.glob(os.path.join(d, "*_counter_collection.csv")):
            for r in csv.DictReader(open(f)):
                key = (short(r["Kernel_Name"]), int(r["Grid_Size"]))
                vals[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return vals


def main(argv):
    argv = list(argv)
    out_json = None
    if "--traffic-json" in argv:
        i = argv.index("--traffic-json")
        out_json = argv[i + 1]
        del argv[i:i + 2]
    if not argv:
        print(__doc__)
        return 1
    trace = load_trace(argv[0])
    pmc = load_pmc(argv[1:])
    # copy calibration: the largest copy dispatch
    copy = [k for k in pmc if k[0] == "__amd_rocclr_copyBuffer"]
    fetch_f = write_f = None
    if copy:
        k = max(copy, key=lambda k: max(pmc[k].get("FETCH_SIZE", [0])))
        fs, ws = max(pmc[k].get("FETCH_SIZE", [0])), max(pmc[k].get("WRITE_SIZE", [0]))
        if fs > 0 and ws > 0:
            fetch_f, write_f = COPY_BYTES / (fs * 1024), COPY_BYTES / (ws * 1024)
            print("calibration: plain copy of 512 MiB reads FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB "
                  "-> HBM read bytes = %.3f x FETCH_SIZE x 1024, write bytes = %.3f x WRITE_SIZE x 1024"
                  % (fs, ws, fetch_f, write_f))
    keys = sorted(set(trace) | set(pmc), key=lambda k: -sum(trace.get(k, [0])))
    for k in keys:
        if k[0].startswith(("__amd_rocclr", "at::native")) and k[0] != "__amd_rocclr_copyBuffer":
            continue
        d = trace.get(k, [])
        line = "%s grid %d: %d dispatches" % (k[0], k[1], len(d))
        if d:
            line += ", mean %.4f ms" % (sum(d) / len(d) / 1e6)
        print(line)
        c = {n: sum(v) / len(v) for n, v in pmc.get(k, {}).items()}
        if not c:
            continue
        print("   " + ", ".join("%s %.4g" % (n, v) for n, v in sorted(c.items())))
        derived = []
        if fetch_f and "FETCH_SIZE" in c:
            derived.append("HBM read %.1f MB" % (c["FETCH_SIZE"] * 1024 * fetch_f / 1e6))
        if write_f and "WRITE_SIZE" in c:
            derived.append("HBM write %.1f MB" % (c["WRITE_SIZE"] * 1024 * write_f / 1e6))
        if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c and c["TCC_HIT_sum"] + c["TCC_MISS_sum"] > 0:
            derived.append("L2 hit %.1f%%" % (100 * c["TCC_HIT_sum"] / (c["TCC_HIT_sum"] + c["TCC_MISS_sum"])))
        if "GRBM_GUI_ACTIVE" in c and "SQ_BUSY_CU_CYCLES" in c:
            cyc = c["GRBM_GUI_ACTIVE"] / 8.0                 # summed over the 8 XCDs
            derived.append("%.0f kernel cycles per XCD" % cyc)
        if "SQ_INSTS_VALU" in c and "SQ_WAVE_CYCLES" in c and c["SQ_WAVE_CYCLES"] > 0:
            derived.append("wait share %.0f%% of wave cycles" % (100 * c.get("SQ_WAIT_INST_ANY", 0) / c["SQ_WAVE_CYCLES"]))
        if "TA_BUSY_avr" in c and "GRBM_GUI_ACTIVE" in c and c["GRBM_GUI_ACTIVE"] > 0:
            derived.append("TA (address unit) busy %.0f%% of kernel cycles"
                           % (100 * c["TA_BUSY_avr"] / (c["GRBM_GUI_ACTIVE"] / 8.0)))
        if "SQ_INSTS_VALU" in c and "GRBM_GUI_ACTIVE" in c and c["GRBM_GUI_ACTIVE"] > 0:
            derived.append("VALU issue %.2f per CU-cycle"
                           % (c["SQ_INSTS_VALU"] / (256 * c["GRBM_GUI_ACTIVE"] / 8.0)))
        if "SQ_INSTS_LDS" in c and c.get("SQ_INSTS_LDS", 0) > 0:
            derived.append("LDS bank-conflict cycles per LDS instruction %.2f"
                           % (c.get("SQ_LDS_BANK_CONFLICT", 0) / c["SQ_INSTS_LDS"]))
        if derived:
            print("   -> " + "; ".join(derived))
    if out_json:
        if not (fetch_f and write_f):
            print("no copy calibration in the counter runs: no traffic summary written")
            return 1
        kernels = {}
        for (name, grid), c in pmc.items():
            if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c or name.startswith(("__amd", "at::")):
                continue
            if name in kernels and kernels[name]["grid"] >= grid:
                continue
            fk = sum(c["FETCH_SIZE"]) / len(c["FETCH_SIZE"])
            wk = sum(c["WRITE_SIZE"]) / len(c["WRITE_SIZE"])
            d = trace.get((name, grid), [])
            kernels[name] = {"grid": grid, "fetch_kib": fk, "write_kib": wk,
                             "read_bytes": fk * 1024 * fetch_f, "write_bytes": wk * 1024 * write_f,
                             "bytes_per_launch": int(fk * 1024 * fetch_f + wk * 1024 * write_f),
                             "mean_ms": sum(d) / len(d) / 1e6 if d else None}
        rec = {"source_hash": source_hash(),
               "calibration": {"copy_bytes": COPY_BYTES, "fetch_factor": fetch_f, "write_factor": write_f},
               "kernels": dict(sorted(kernels.items()))}
        with open(out_json, "w") as f:
            json.dump(rec, f, indent=1)
        print("wrote %s (%d kernels)" % (out_json, len(kernels)))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
