"""Short text summaries of rocprofv3 output (kernel traces and counter runs).

    python -m paper_2410_15519_amd.profsum trace DB TITLE CMD > summary.md
    python -m paper_2410_15519_amd.profsum pmc FETCH_CSV WRITE_CSV COPY_MIB TITLE CMD > summary.md
    python -m paper_2410_15519_amd.profsum mfma COUNTER_CSV CUS TITLE CMD > summary.md
    python -m paper_2410_15519_amd.profsum counters CSV[:CSV...] PREFIXES TITLE CMD > summary.md

`trace` groups the kernel records of a rocpd database by kernel name and
grid.  `pmc` averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per kernel
over two counter runs of the same command, scales each by what the counter
reads for the plain copy kernel k_copy16 of COPY_MIB MiB, and prints the
HBM traffic per launch of every kernel with the sha256 of the kernel source
it was taken on (a reader of the summary can tell when the kernels changed).
`mfma` reports the MFMA busy fraction and the executed MFMA flops per kernel
from one counter run (see `mfma`).
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hip")


def kernel_source_sha() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def short_name(name: str) -> str:
    name = name.replace("ctd::", "").replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*$", "", name)
    return name.replace("void ", "").strip()


def trace(db: str, title: str, cmd: str) -> str:
    """Kernel records grouped by name and grid.  Launches of a sweep that was
    enqueued ahead of the host's decision and returned at once (its mode had
    ended) are counted apart: within a group, a launch shorter than a quarter
    of the group's median is such a launch, and `avg us (ran)` is the mean of
    the others."""
    con = sqlite3.connect(db)
    groups = collections.defaultdict(list)
    meta = {}
    for r in con.execute("select name, grid_x, grid_y, workgroup_x, duration, lds_size, vgpr_count, "
                         "accum_vgpr_count, scratch_size from kernels"):
        k = (r[0], r[1], r[2])
        groups[k].append(r[4] / 1000.0)
        meta[k] = (r[3], r[5], r[6], r[7], r[8])
    total = sum(sum(v) for v in groups.values()) / 1e3
    rows = []
    for k, d in groups.items():
        d.sort()
        med = d[len(d) // 2]
        ran = [x for x in d if x >= 0.25 * med]
        rows.append((k, len(d), len(d) - len(ran), sum(d) / len(d), sum(ran) / max(1, len(ran)),
                     d[0], d[-1], sum(d) / 1e3))
    rows.sort(key=lambda r: -r[7])
    out = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "",
           "```", cmd, "```", "",
           "Summary of the rocpd database it wrote: kernel records grouped by name and grid "
           "(grid in work-items, durations in microseconds).  `returned` counts the launches of "
           "speculatively enqueued sweeps that returned at once (shorter than a quarter of the "
           "group's median); `avg us (ran)` averages the other launches.", "",
           f"Total kernel time in the trace: {total:.1f} ms", "",
           "| kernel | grid (x, y) | wg | launches | returned | avg us | avg us (ran) | min us | max us | total ms | LDS B | VGPR | AGPR | scratch |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, n, nret, avg, avg_ran, mn, mx, tot in rows[:18]:
        wg, lds, vg, ag, sc = meta[k]
        out.append(f"| {short_name(k[0])} | ({k[1]}, {k[2]}) | {wg} | {n} | {nret} | {avg:.1f} | {avg_ran:.1f} | "
                   f"{mn:.1f} | {mx:.1f} | {tot:.1f} | {lds} | {vg} | {ag} | {sc} |")
    by_name = collections.defaultdict(lambda: [0, 0.0])
    for (name, _, _), d in groups.items():
        by_name[short_name(name)][0] += len(d)
        by_name[short_name(name)][1] += sum(d) / 1e3
    out += ["", "All grids of a kernel together:", "",
            "| kernel | launches | avg us | total ms |", "|---|---|---|---|"]
    for name, (n, tot) in sorted(by_name.items(), key=lambda kv: -kv[1][1])[:20]:
        out.append(f"| {name} | {n} | {1e3 * tot / max(1, n):.1f} | {tot:.1f} |")
    return "\n".join(out) + "\n"


def _per_kernel(path: str, counter: str):
    """{kernel [grid]: (dispatches, mean counter value per dispatch)} from a
    counter CSV; one entry per kernel name and grid size (work-items)."""
    acc = collections.defaultdict(float)
    disp = collections.defaultdict(set)
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = short_name(row.get("Kernel_Name", ""))
            k = name if name == "k_copy16" else f"{name} [{row.get('Grid_Size', '?')}]"
            acc[k] += float(row["Counter_Value"])
            disp[k].add(row.get("Dispatch_Id", row.get("Correlation_Id", "")))
    return {k: (len(disp[k]), acc[k] / max(1, len(disp[k]))) for k in acc}


def pmc(fetch_csv: str, write_csv: str, copy_mib: float, title: str, cmd: str) -> str:
    fe = _per_kernel(fetch_csv, "FETCH_SIZE")
    wr = _per_kernel(write_csv, "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0
    if "k_copy16" not in fe or "k_copy16" not in wr:
        raise SystemExit("no k_copy16 dispatch in the counter runs")
    f_scale = copy_kib / fe["k_copy16"][1]
    w_scale = copy_kib / wr["k_copy16"][1]
    names = sorted(set(fe) & set(wr), key=lambda k: -(fe[k][0] * (fe[k][1] + wr[k][1])))
    out = [f"# {title}", "", "Commands (run from the repository root on one MI355X, one counter per run):",
           "", "```", cmd, "```", "",
           f"Counter values are KiB per dispatch, averaged per kernel name and grid size.  Scale: the plain copy "
           f"kernel k_copy16 of {copy_mib:g} MiB reads FETCH_SIZE {fe['k_copy16'][1]:.0f} KiB and "
           f"WRITE_SIZE {wr['k_copy16'][1]:.0f} KiB, so FETCH_SIZE x {f_scale:.4f} and WRITE_SIZE x "
           f"{w_scale:.4f} give bytes moved to and from HBM.", "",
           f"kernel source sha256 (first 16 hex): {kernel_source_sha()}", "",
           "| kernel [grid work-items] | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read MB | HBM write MB | traffic MB/launch |",
           "|---|---|---|---|---|---|---|"]
    for k in names[:16]:
        rd = fe[k][1] * f_scale * 1024 / 1e6
        wt = wr[k][1] * w_scale * 1024 / 1e6
        out.append(f"| {k} | {fe[k][0]} | {fe[k][1]:.1f} | {wr[k][1]:.1f} | {rd:.3f} | {wt:.3f} | {rd + wt:.3f} |")
    out.append("")
    for k in names:
        tb = (fe[k][1] * f_scale + wr[k][1] * w_scale) * 1024
        out.append(f"traffic_bytes_per_launch {k} = {tb:.0f}")
    return "\n".join(out) + "\n"


def traffic_from_summary(path: str, kernel: str):
    """Traffic per launch recorded for `kernel` ("name [grid]"), or None when
    the summary is missing or was taken on a different kernel source."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel source sha256 \(first 16 hex\): (\w+)", text)
    if not m or m.group(1) != kernel_source_sha():
        return None
    m = re.search(r"^traffic_bytes_per_launch " + re.escape(kernel) + r" = (\d+)$", text, flags=re.M)
    return float(m.group(1)) if m else None


def mfma(csv_path: str, cus: int, title: str, cmd: str, xcds: int = 8, simds: int = 4) -> str:
    """MFMA activity per kernel and grid from one counter run holding
    SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE, SQ_INSTS_VALU_MFMA_MOPS_F32 and
    SQ_INSTS_VALU_MFMA_MOPS_F64 (per-dispatch means).  GRBM_GUI_ACTIVE reads
    the sum over the XCDs; the MFMA busy cycles are summed over all SIMDs (32
    per executed 16x16x4 FP32 MFMA).  Busy fraction = busy cycles /
    (GRBM_GUI_ACTIVE / xcds x cus x simds); executed flops = MOPS count x 512."""
    busy = _per_kernel(csv_path, "SQ_VALU_MFMA_BUSY_CYCLES")
    act = _per_kernel(csv_path, "GRBM_GUI_ACTIVE")
    m32 = _per_kernel(csv_path, "SQ_INSTS_VALU_MFMA_MOPS_F32")
    m64 = _per_kernel(csv_path, "SQ_INSTS_VALU_MFMA_MOPS_F64")
    names = sorted((k for k in busy if k in act and (m32.get(k, (0, 0))[1] + m64.get(k, (0, 0))[1]) > 0),
                   key=lambda k: -busy[k][0] * busy[k][1])
    out = [f"# {title}", "", "Commands (run from the repository root on one MI355X):", "", "```", cmd, "```", "",
           f"Per-dispatch means per kernel name and grid size.  GRBM_GUI_ACTIVE is the sum over the {xcds} "
           f"XCDs and the MFMA busy cycles the sum over the {cus * simds} SIMDs (32 per executed 16x16x4 "
           f"FP32 MFMA), so MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {xcds} x "
           f"{cus * simds}); executed flops = SQ_INSTS_VALU_MFMA_MOPS_* x 512.", "",
           f"kernel source sha256 (first 16 hex): {kernel_source_sha()}", "",
           "| kernel [grid work-items] | dispatches | GRBM_GUI_ACTIVE | MFMA busy cycles | MFMA busy | executed FP32 MFMA GFLOP | executed FP64 MFMA GFLOP |",
           "|---|---|---|---|---|---|---|"]
    for k in names[:16]:
        n, b = busy[k]
        a = act[k][1]
        f32 = m32.get(k, (0, 0.0))[1] * 512 / 1e9
        f64 = m64.get(k, (0, 0.0))[1] * 512 / 1e9
        frac = b / (a / xcds * cus * simds) if a > 0 else 0.0
        out.append(f"| {k} | {n} | {a:.0f} | {b:.0f} | {100 * frac:.1f} % | {f32:.3f} | {f64:.3f} |")
    return "\n".join(out) + "\n"


def counters(csv_paths, prefixes, title: str, cmd: str) -> str:
    """Every counter of one or more counter runs, per-dispatch means per
    kernel name and grid, for the kernels whose name starts with one of
    `prefixes` (comma-separated), with the ratios used to read them: VALU
    and LDS instructions per wave, LDS bank-conflict cycles per LDS
    instruction, and the share of wave cycles spent waiting."""
    vals = collections.defaultdict(dict)
    disp = {}
    names = set()
    for path in csv_paths:
        with open(path) as f:
            for row in csv.DictReader(f):
                names.add(row.get("Counter_Name"))
    for path in csv_paths:
        for c in sorted(n for n in names if n):
            for k, (nd, v) in _per_kernel(path, c).items():
                if any(k.startswith(p) for p in prefixes.split(",")):
                    vals[k][c] = v
                    disp[k] = nd
    cols = sorted({c for v in vals.values() for c in v})
    out = [f"# {title}", "", "Commands (run from the repository root on one MI355X):", "", "```", cmd, "```", "",
           "Per-dispatch means per kernel name and grid size (counters summed over the device).", "",
           f"kernel source sha256 (first 16 hex): {kernel_source_sha()}", "",
           "| kernel [grid work-items] | dispatches | " + " | ".join(cols) + " |",
           "|---|---|" + "---|" * len(cols)]
    for k in sorted(vals, key=lambda k: -disp[k]):
        out.append(f"| {k} | {disp[k]} | " + " | ".join(f"{vals[k].get(c, float('nan')):.4g}" for c in cols) + " |")
    out += ["", "Ratios:", "", "| kernel | VALU/wave | LDS/wave | bank-conflict cycles per LDS inst | "
            "wait / wave cycles | busy / wave cycles (VALU) |", "|---|---|---|---|---|---|"]
    for k in sorted(vals, key=lambda k: -disp[k]):
        v = vals[k]
        w = v.get("SQ_WAVES", 0.0)
        def r(a, b):
            return f"{v[a] / v[b]:.3g}" if a in v and b in v and v[b] else "-"
        valu = f"{v['SQ_INSTS_VALU'] / w:.0f}" if "SQ_INSTS_VALU" in v and w else "-"
        lds = f"{v['SQ_INSTS_LDS'] / w:.0f}" if "SQ_INSTS_LDS" in v and w else "-"
        out.append(f"| {k} | {valu} | {lds} | {r('SQ_LDS_BANK_CONFLICT', 'SQ_INSTS_LDS')} | "
                   f"{r('SQ_WAIT_INST_ANY', 'SQ_WAVE_CYCLES')} | {r('SQ_ACTIVE_INST_VALU', 'SQ_WAVE_CYCLES')} |")
    return "\n".join(out) + "\n"


def main(argv):
    if len(argv) >= 4 and argv[0] == "trace":
        sys.stdout.write(trace(argv[1], argv[2], argv[3]))
    elif len(argv) >= 6 and argv[0] == "pmc":
        sys.stdout.write(pmc(argv[1], argv[2], float(argv[3]), argv[4], argv[5]))
    elif len(argv) >= 5 and argv[0] == "mfma":
        sys.stdout.write(mfma(argv[1], int(argv[2]), argv[3], argv[4]))
    elif len(argv) >= 5 and argv[0] == "counters":
        sys.stdout.write(counters(argv[1].split(":"), argv[2], argv[3], argv[4]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
