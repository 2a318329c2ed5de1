"""Summaries of rocprofv3 output for the records kept under ``profiles/``.

Three commands (run from the repository root):

``python -m paper_2511_16576_amd.profiling stats --csv <kernel_stats.csv> --out <file.md> --title T --command C``
    Markdown table of a ``--kernel-trace --stats`` run (per-kernel calls,
    average / min / max duration, share of GPU time).

``python -m paper_2511_16576_amd.profiling valu --pmc <counter_collection.csv> --stats <kernel_stats.csv> --out <file.md> --command C``
    Issued VALU work per dispatch (``SQ_INSTS_VALU`` x 64 lanes) over the
    kernel's average duration from the trace run, against the VALU peak of
    256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.

``python -m paper_2511_16576_amd.profiling window --trace <kernel_trace.csv> --replays R --out <file.md> --title T --command C``
    Per-replay kernel table of the dispatches between two marker kernels
    (torch's ``spin_kernel``; ``bench.py --trace-window m1,m2,..`` puts R
    replays of each method's captured query batch between consecutive
    markers; ``--index i`` picks window i), so the benchmark's setup (data
    generation, training, brute force) stays out.

``python -m paper_2511_16576_amd.profiling traffic --fetch <counter_collection.csv> --write <counter_collection.csv> --out <file.json> --md <file.md> --command-fetch C1 --command-write C2 [--window i --kernels k1,k2 --title T]``
    HBM traffic per dispatch of the hot kernels from one ``--pmc FETCH_SIZE``
    and one ``--pmc WRITE_SIZE`` run.  Both runs include one device-to-device
    copy of a known size (``bench.py --copy-calibration``: 256 MiB); each
    counter is scaled by (copy bytes) / (what that counter reads for the copy
    dispatch), so the result is in bytes moved.  The JSON also records a hash
    of each kernel's sources: a reader (``bench.py``) uses the figure only
    while the kernel is unchanged.  ``--window i`` keeps the dispatches
    between marker kernels i and i + 1 (as ``window``).

``python -m paper_2511_16576_amd.profiling mfma --pmc <counter_collection.csv> --trace <kernel_trace.csv> --replays R --window i --out <file.md> --command C``
    BF16 matrix-core work and busy cycles per dispatch of the kernels in
    window i, against the dense BF16 peak.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
COPY_BYTES = 256 << 20

# kernel -> the sources it is built from
KERNEL_SOURCES = {
    "k_refine": ["refine.hip", "internal.hpp"],
    "k_sign": ["sign.hip", "sign_common.hpp", "internal.hpp"],
    "k_bin_lookup": ["binned.hip", "sign_common.hpp", "internal.hpp"],
    "k_rank_jhat_sort": ["rank.hip", "internal.hpp"],
    "k_rank_jhat_packed": ["rank.hip", "internal.hpp"],
    "k_sparse": ["query.hip", "internal.hpp"],
    "k_sparse_sort": ["query.hip", "internal.hpp"],
    "k_sparse_sort_big": ["query.hip", "internal.hpp"],
    "k_refine_wide": ["refine.hip", "internal.hpp"],
    "k_score_pairs": ["score.hip", "scorer_common.hpp", "internal.hpp"],
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    if "(anonymous namespace)::" in name:
        name = name.split("(anonymous namespace)::")[1]
    name = name.split("(")[0].replace("void ", "")
    if name.startswith("k_sign"):
        return "k_sign"
    return name


def stats_markdown(csv_path: str, title: str, command: str, notes: str = "", top: int = 18) -> str:
    rows = list(csv.DictReader(open(csv_path)))
    out = [f"# {title}", "", "Command (from `/tmp` with `TMPDIR=/tmp`; `<repo>` is the repository root):", "",
           "```", command, "```", ""]
    if notes:
        out += [notes, ""]
    out += ["| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        nm = r["Name"]
        if "(anonymous namespace)::" in nm:
            nm = nm.split("(anonymous namespace)::")[1]
        nm = nm.split("(")[0].replace("void ", "")
        out.append(f"| {nm} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def _window_rows(rows, start_key, name_key, index=0, marker="spin_kernel"):
    """Rows strictly between marker dispatches `index` and `index + 1`
    (windows are numbered in time order)."""
    rows = sorted(rows, key=lambda r: int(r[start_key]))
    idx = [i for i, r in enumerate(rows) if marker in r[name_key]]
    if len(idx) < index + 2:
        raise RuntimeError(f"fewer than {index + 2} {marker} dispatches: no window {index}")
    return rows[idx[index] + 1:idx[index + 1]]


def window_markdown(trace_csv: str, replays: int, title: str, command: str, notes: str = "", index: int = 0) -> str:
    rows = _window_rows(list(csv.DictReader(open(trace_csv))), "Start_Timestamp", "Kernel_Name", index)
    per = collections.defaultdict(list)
    for r in rows:
        per[short_name(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    busy = sum(sum(v) for v in per.values())
    span = int(rows[-1]["End_Timestamp"]) - int(rows[0]["Start_Timestamp"]) if rows else 0
    out = [f"# {title}", "", "Command (from `/tmp` with `TMPDIR=/tmp`; `<repo>` is the repository root):", "",
           "```", command, "```", ""]
    if notes:
        out += [notes, ""]
    out += [f"{replays} replays between the marker kernels: {len(rows)} dispatches, GPU busy "
            f"{busy / 1e6 / replays:.3f} ms and first start to last end {span / 1e6 / replays:.3f} ms per replay.", "",
            "| kernel | dispatches per replay | avg us | min us | max us | us per replay | % of busy |",
            "|---|---|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| {k} | {len(v) / replays:g} | {sum(v) / len(v) / 1e3:.1f} | {min(v) / 1e3:.1f} | "
                   f"{max(v) / 1e3:.1f} | {sum(v) / replays / 1e3:.1f} | {100.0 * sum(v) / max(busy, 1):.2f} |")
    return "\n".join(out) + "\n"


def _counter_rows(csv_path: str, window: int | None):
    rows = list(csv.DictReader(open(csv_path)))
    if window is None:
        return rows
    # dispatches between marker kernels `window` and `window + 1`, in
    # dispatch order (every dispatch has one row per counter)
    order = sorted({int(r["Dispatch_Id"]) for r in rows})
    name = {int(r["Dispatch_Id"]): r["Kernel_Name"] for r in rows}
    marks = [d for d in order if "spin_kernel" in name[d]]
    if len(marks) < window + 2:
        raise RuntimeError(f"fewer than {window + 2} marker dispatches: no window {window}")
    lo, hi = marks[window], marks[window + 1]
    return [r for r in rows if lo < int(r["Dispatch_Id"]) < hi]


def _per_kernel(csv_path: str, counter: str, window: int | None = None, copies_from: str | None = None):
    """kernel short name -> list of per-dispatch counter values (KiB), and
    the values of the copy dispatches (over the whole run)."""
    per = collections.defaultdict(list)
    copies = []
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]:
            copies.append(float(r["Counter_Value"]))
    for r in _counter_rows(csv_path, window):
        if r["Counter_Name"] != counter:
            continue
        per[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return per, copies


def traffic(fetch_csv: str, write_csv: str, kernels=("k_refine", "k_sign"), window: int | None = None) -> dict:
    fetch, fcopies = _per_kernel(fetch_csv, "FETCH_SIZE", window)
    write, wcopies = _per_kernel(write_csv, "WRITE_SIZE", window)
    if not fcopies or not wcopies:
        raise RuntimeError("no copy dispatch in the counter runs (run bench.py with --copy-calibration)")
    # the calibration copy is the largest copy dispatch of each run
    f_copy, w_copy = max(fcopies), max(wcopies)
    f_scale = COPY_BYTES / (f_copy * 1024.0)
    w_scale = COPY_BYTES / (w_copy * 1024.0)
    out = {"copy_bytes": COPY_BYTES, "fetch_kib_for_copy": f_copy, "write_kib_for_copy": w_copy,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}}
    for k in kernels:
        fv, wv = fetch.get(k, []), write.get(k, [])
        if not fv or not wv:
            continue
        f_kib, w_kib = sum(fv) / len(fv), sum(wv) / len(wv)
        out["kernels"][k] = {
            "dispatches": len(fv), "fetch_kib": f_kib, "write_kib": w_kib,
            "fetch_bytes": f_kib * 1024.0 * f_scale, "write_bytes": w_kib * 1024.0 * w_scale,
            "bytes": f_kib * 1024.0 * f_scale + w_kib * 1024.0 * w_scale,
            "source_hash": source_hash(k),
        }
    return out


def traffic_markdown(t: dict, cmd_fetch: str, cmd_write: str,
                     title: str = "HBM traffic per dispatch of the hot kernels (workload 2 bench step)") -> str:
    out = [f"# {title}", "",
           "Commands (from `/tmp` with `TMPDIR=/tmp`; `<repo>` is the repository root):", "", "```",
           cmd_fetch, cmd_write, "```", "",
           f"Calibration: a {t['copy_bytes'] >> 20} MiB device-to-device copy reads as "
           f"FETCH_SIZE = {t['fetch_kib_for_copy']:.1f} KiB and WRITE_SIZE = {t['write_kib_for_copy']:.1f} KiB, "
           f"so FETCH_SIZE is scaled by {t['fetch_scale']:.4f} and WRITE_SIZE by {t['write_scale']:.4f} "
           "to give bytes.", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes read | bytes written | total | source hash |",
           "|---|---|---|---|---|---|---|---|"]
    for k, v in t["kernels"].items():
        out.append(f"| {k} | {v['dispatches']} | {v['fetch_kib']:.1f} | {v['write_kib']:.1f} | "
                   f"{v['fetch_bytes'] / 1e6:.1f} MB | {v['write_bytes'] / 1e6:.1f} MB | {v['bytes'] / 1e6:.1f} MB | "
                   f"`{v['source_hash']}` |")
    return "\n".join(out) + "\n"


PEAK_LANE_CYCLES = 256 * 4 * 16 * 2.4e9


def valu_markdown(pmc_csv: str, stats_csv: str, command: str, kernels=("k_refine", "k_sign")) -> str:
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(pmc_csv)):
        per[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = {}
    for r in csv.DictReader(open(stats_csv)):
        dur.setdefault(short_name(r["Name"]), float(r["AverageNs"]) * 1e-9)
    out = ["# Issued VALU work of the hot kernels (workload 2 bench step)", "",
           "Command (from `/tmp` with `TMPDIR=/tmp`; `<repo>` is the repository root):", "", "```", command,
           "```", "",
           "Hardware VALU fraction = SQ_INSTS_VALU x 64 lane-cycles / average duration (kernel-trace run) / "
           "39.3 T lane-cycles/s.  It counts every issued VALU instruction, useful or not; the bench's "
           "`roofline.frac` counts only the algorithmic operations.", "",
           "| kernel | dispatches | VALU instr / dispatch | SALU instr / dispatch | waves / dispatch | avg duration ms | "
           "issued T lane-cycles/s | hardware VALU fraction |", "|---|---|---|---|---|---|---|---|"]
    for k in kernels:
        d = per.get(k)
        if not d or k not in dur:
            continue
        mean = {c: sum(v) / len(v) for c, v in d.items()}
        valu = mean.get("SQ_INSTS_VALU", 0.0)
        rate = valu * 64 / dur[k]
        out.append(f"| {k} | {len(d['SQ_INSTS_VALU'])} | {valu:.4g} | {mean.get('SQ_INSTS_SALU', 0):.4g} | "
                   f"{mean.get('SQ_WAVES', 0):.4g} | {dur[k] * 1e3:.3f} | {rate / 1e12:.2f} | "
                   f"{rate / PEAK_LANE_CYCLES:.3f} |")
    return "\n".join(out) + "\n"


PEAK_BF16_FLOPS = 2.5e15


def mfma_markdown(pmc_csv: str, trace_csv: str, command: str, replays: int, window: int | None = None,
                  title: str = "Matrix-core use of the scorer kernels") -> str:
    """Per kernel: BF16 MFMA operations (SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512)
    and busy cycles per dispatch from a counter run; durations from the
    windowed kernel trace of the same command."""
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in _counter_rows(pmc_csv, window):
        per[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = collections.defaultdict(list)
    trows = list(csv.DictReader(open(trace_csv)))
    if window is not None:
        trows = _window_rows(trows, "Start_Timestamp", "Kernel_Name", window)
    for r in trows:
        dur[short_name(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    out = [f"# {title}", "", "Commands (from `/tmp` with `TMPDIR=/tmp`; `<repo>` is the repository root):", "",
           "```", command, "```", "",
           "BF16 FLOP per dispatch = SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512 (the counter's definition); achieved = "
           "FLOP / average duration (kernel trace of the same command) against the dense BF16 peak of "
           f"{PEAK_BF16_FLOPS / 1e15:.1f} PFLOP/s.", "",
           "| kernel | dispatches | BF16 GFLOP / dispatch | avg duration us | achieved TFLOP/s | fraction of peak |",
           "|---|---|---|---|---|---|"]
    for k, d in sorted(per.items()):
        mops = d.get("SQ_INSTS_VALU_MFMA_MOPS_BF16")
        if not mops or sum(mops) == 0 or k not in dur:
            continue
        flops = sum(mops) / len(mops) * 512
        t = sum(dur[k]) / len(dur[k])
        out.append(f"| {k} | {len(mops)} | {flops / 1e9:.3f} | {t * 1e6:.1f} | {flops / t / 1e12:.1f} | "
                   f"{flops / t / PEAK_BF16_FLOPS:.4f} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--notes", default="")
    v = sub.add_parser("valu")
    v.add_argument("--pmc", required=True)
    v.add_argument("--stats", required=True)
    v.add_argument("--out", required=True)
    v.add_argument("--command", required=True)
    w = sub.add_parser("window")
    w.add_argument("--trace", required=True)
    w.add_argument("--replays", type=int, required=True)
    w.add_argument("--out", required=True)
    w.add_argument("--title", required=True)
    w.add_argument("--command", required=True)
    w.add_argument("--notes", default="")
    w.add_argument("--index", type=int, default=0, help="window number (time order)")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--md", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--window", type=int, default=None, help="window number (marker kernels)")
    t.add_argument("--kernels", default="k_refine,k_sign")
    t.add_argument("--title", default="HBM traffic per dispatch of the hot kernels (workload 2 bench step)")
    m = sub.add_parser("mfma")
    m.add_argument("--pmc", required=True)
    m.add_argument("--trace", required=True)
    m.add_argument("--replays", type=int, required=True)
    m.add_argument("--window", type=int, default=None)
    m.add_argument("--title", default="Matrix-core use of the scorer kernels")
    m.add_argument("--out", required=True)
    m.add_argument("--command", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        open(a.out, "w").write(stats_markdown(a.csv, a.title, a.command, a.notes))
    elif a.cmd == "window":
        open(a.out, "w").write(window_markdown(a.trace, a.replays, a.title, a.command, a.notes, a.index))
    elif a.cmd == "valu":
        open(a.out, "w").write(valu_markdown(a.pmc, a.stats, a.command))
    elif a.cmd == "mfma":
        open(a.out, "w").write(mfma_markdown(a.pmc, a.trace, a.command, a.replays, a.window, a.title))
    else:
        res = traffic(a.fetch, a.write, tuple(a.kernels.split(",")), a.window)
        json.dump(res, open(a.out, "w"), indent=1)
        open(a.md, "w").write(traffic_markdown(res, a.command_fetch, a.command_write, a.title))


if __name__ == "__main__":
    main()
