"""Summarise rocprofv3 CSV output of a bench run into a short text file.

Inputs are the directories written by three rocprofv3 runs of the same
command: one with ``--kernel-trace --stats``, one with ``--pmc FETCH_SIZE``
and one with ``--pmc WRITE_SIZE`` (all with ``--output-format csv``). The
command is expected to start with one plain device-to-device copy of a known
size (``bench.py --calib-copy-mb``); the byte counters of every other
dispatch are scaled by (copy bytes) / (counter value of that copy), so the
summary reports bytes rather than the counters' own units.

A kernel group is named as ``label=regex@last`` : the dispatches whose name
matches ``regex``, of which the last ``last`` (the timed step of a bench run
whose warm-up and autotuning dispatches come first) are averaged.

    python -m paper_2403_18661_amd.profsum --trace DIR --fetch DIR --write DIR \\
        --calib-mb 1024 --group 'f32=conv_mfma_kernel<afm::PF32,@280' --cmd '...' --out FILE

A launch sequence is named as ``label=regex@start:count``: the ``count``
consecutive dispatches matching ``regex`` from position ``start`` (negative:
from the end) of the matches, one row each; e.g. the 35 conv launches of one
8192-window batch, layer by layer.  The counter runs are separate processes,
so their dispatches are matched to the trace's by position; a row whose
kernel differs between the runs (an autotuner that chose another tile) is
marked.

Optional ``--sq DIR`` runs (``--pmc`` with SQ_* counters, as many as one
pass collects) add, per group, each counter summed over the group's
dispatches and divided by their number.

The summary ends with the kernel sources its figures depend on
(``--sources``, default: all of them) and their ``source_sha256``, so that a
reader of the figures can tell whether those kernels changed since.
"""
import argparse
import csv
import hashlib
import os
import re

KERNEL_SOURCES = ("csrc/net_kernels.h", "csrc/gn_kernels.h", "csrc/net.hip", "csrc/fused_tiny.h", "csrc/whiten.hip", "csrc/psd.hip",
                  "csrc/fft_lds.h", "csrc/tables.hip", "csrc/common.h")


def source_sha256(sources=KERNEL_SOURCES):
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for rel in sources:
        with open(os.path.join(here, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _rows(d, suffix):
    names = [n for n in os.listdir(d) if n.endswith(suffix)]
    if not names:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    with open(os.path.join(d, names[0])) as f:
        return list(csv.DictReader(f))


def _seqs(specs):
    out = []
    for s in specs:
        label, rest = s.split("=", 1)
        rx, rng = rest.rsplit("@", 1)
        start, count = (int(v) for v in rng.split(":"))
        if count < 1:
            raise ValueError(f"{s}: count must be positive")
        out.append((label, re.compile(rx), start, count))
    return out


def _slice(rows, rx, start, count):
    sel = [r for r in rows if rx.search(r["Kernel_Name"])]
    end = start + count
    got = sel[start:end if end != 0 else None]
    if len(got) != count:
        raise ValueError(f"{rx.pattern}: {len(sel)} dispatches, no {count} from position {start}")
    return got


def _short(name):
    m = re.search(r"<(.*)>\(", name)
    return re.sub(r"afm::|\s", "", m.group(1)) if m else name[:60]


def _groups(specs):
    out = []
    for s in specs:
        label, rest = s.split("=", 1)
        rx, last = rest.rsplit("@", 1)
        out.append((label, re.compile(rx), int(last)))
    return out


def _pick(rows, rx, last):
    sel = [r for r in rows if rx.search(r["Kernel_Name"])]
    if len(sel) < last:
        raise ValueError(f"{rx.pattern}: {len(sel)} dispatches, wanted the last {last}")
    return sel[-last:]


def _calib(rows, calib_bytes):
    copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
    if not copies:
        raise ValueError("no copy dispatch to calibrate against")
    big = max(copies, key=lambda r: float(r["Counter_Value"]))
    return calib_bytes / (float(big["Counter_Value"]) * 1024.0), float(big["Counter_Value"])


def summarise(trace, fetch, write, calib_mb, groups, cmd, top=12, sq_dirs=(), sources=KERNEL_SOURCES, seqs=()):
    calib_bytes = calib_mb * 2 ** 20
    kt = _rows(trace, "kernel_trace.csv")
    ks = _rows(trace, "kernel_stats.csv")
    if not ks:
        raise ValueError(f"{trace}: kernel_stats.csv holds no rows (profiler output not yet complete)")
    fr = _rows(fetch, "counter_collection.csv")
    wr = _rows(write, "counter_collection.csv")
    kf, f_raw = _calib(fr, calib_bytes)
    kw, w_raw = _calib(wr, calib_bytes)
    lines = ["# rocprofv3 summary", "", "command:", "  " + cmd.replace("\n", "\n  "), ""]
    lines.append(f"byte-counter calibration: plain copy of {calib_mb} MiB reads FETCH_SIZE {f_raw:.1f} KiB "
                 f"(factor {kf:.4f}) and WRITE_SIZE {w_raw:.1f} KiB (factor {kw:.4f})")
    lines.append("")
    lines.append("groups (last N dispatches of the run; durations from --kernel-trace, bytes = counter KiB x "
                 "1024 x factor):")
    lines.append(f"  {'label':10s} {'N':>5s} {'avg_ms':>9s} {'fetch_MB':>10s} {'write_MB':>10s} "
                 f"{'traffic_bytes_per_launch':>26s}")
    for label, rx, last in groups:
        t = _pick(kt, rx, last)
        dur = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in t) / last * 1e-6
        fb = sum(float(r["Counter_Value"]) for r in _pick(fr, rx, last)) * 1024 * kf / last
        wb = sum(float(r["Counter_Value"]) for r in _pick(wr, rx, last)) * 1024 * kw / last
        lines.append(f"  {label:10s} {last:5d} {dur:9.4f} {fb / 1e6:10.2f} {wb / 1e6:10.2f} {fb + wb:26.0f}")
    for d in sq_dirs:
        rows = _rows(d, "counter_collection.csv")
        lines.append("")
        lines.append(f"SQ counters per dispatch ({os.path.basename(os.path.normpath(d))}):")
        for label, rx, last in groups:
            sel = [r for r in rows if rx.search(r["Kernel_Name"])]
            ids = sorted({r["Dispatch_Id"] for r in sel}, key=int)[-last:]
            agg = {}
            for r in sel:
                if r["Dispatch_Id"] in ids:
                    agg[r["Counter_Name"]] = agg.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            vals = "  ".join(f"{k} {v / len(ids):.4g}" for k, v in sorted(agg.items()))
            lines.append(f"  {label:10s} {vals}")
    for label, rx, start, count in seqs:
        t, f, w = (_slice(rows, rx, start, count) for rows in (kt, fr, wr))
        lines.append("")
        lines.append(f"launch sequence {label} ({count} dispatches matching {rx.pattern} from position {start}; "
                     "bytes as above; * = another kernel in a counter run):")
        lines.append(f"  {'#':>3s} {'ms':>8s} {'fetch_MB':>9s} {'write_MB':>9s} {'GB/s':>7s}  kernel")
        for i, (rt, rf, rw) in enumerate(zip(t, f, w)):
            dur = (int(rt["End_Timestamp"]) - int(rt["Start_Timestamp"])) * 1e-6
            fb = float(rf["Counter_Value"]) * 1024 * kf
            wb = float(rw["Counter_Value"]) * 1024 * kw
            mark = "" if rt["Kernel_Name"] == rf["Kernel_Name"] == rw["Kernel_Name"] else " *"
            lines.append(f"  {i + 1:3d} {dur:8.4f} {fb / 1e6:9.2f} {wb / 1e6:9.2f} {(fb + wb) / dur * 1e-6:7.0f}  "
                         f"{_short(rt['Kernel_Name'])}{mark}")
    lines.append("")
    lines.append(f"--stats, top {top} kernels by total time (all dispatches of the run, incl. autotuning):")
    ks = sorted(ks, key=lambda r: -float(r["TotalDurationNs"]))[:top]
    for r in ks:
        lines.append(f"  {float(r['Percentage']):6.2f}%  calls {int(r['Calls']):5d}  avg "
                     f"{float(r['AverageNs']) * 1e-6:8.4f} ms  {r['Name'][:110]}")
    lines.append("")
    lines.append("source_files " + " ".join(sources))
    lines.append(f"source_sha256 {source_sha256(sources)}")
    return "\n".join(lines) + "\n"


def read_traffic(path):
    """{label: bytes per launch} from a summary, or {} if the kernel sources
    changed since it was written (or it does not exist)."""
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return {}
    m = re.search(r"^source_sha256 (\w+)", text, re.M)
    f = re.search(r"^source_files (.+)$", text, re.M)
    sources = tuple(f.group(1).split()) if f else KERNEL_SOURCES
    if not m or not set(sources) <= set(KERNEL_SOURCES) or m.group(1) != source_sha256(sources):
        return {}
    out = {}
    block = text.split("groups (", 1)[1].split("\n\n", 1)[0].splitlines()[2:]
    for ln in block:
        p = ln.split()
        out[p[0]] = {"n": int(p[1]), "avg_ms": float(p[2]), "traffic": float(p[5])}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--calib-mb", type=int, required=True)
    ap.add_argument("--group", action="append", required=True)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--sq", action="append", default=[], help="directory of a --pmc run of SQ counters")
    ap.add_argument("--seq", action="append", default=[], help="label=regex@start:count, one row per dispatch")
    ap.add_argument("--sources", nargs="+", default=list(KERNEL_SOURCES),
                    help="kernel sources (relative to the package) the profiled kernels are built from")
    a = ap.parse_args()
    unknown = set(a.sources) - set(KERNEL_SOURCES)
    if unknown:
        ap.error(f"not kernel sources: {sorted(unknown)}")
    text = summarise(a.trace, a.fetch, a.write, a.calib_mb, _groups(a.group), a.cmd, sq_dirs=a.sq,
                     sources=tuple(a.sources), seqs=_seqs(a.seq))
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
