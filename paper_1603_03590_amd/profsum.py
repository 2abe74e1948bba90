"""Summaries of rocprofv3 CSV output for the measurement records.

``python -m paper_1603_03590_amd.profsum trace <dir> [--after REGEX]`` prints a
markdown table of per-kernel dispatch counts and durations from
``<dir>/run_kernel_trace.csv``.

``python -m paper_1603_03590_amd.profsum util <dir>`` prints the mean per
dispatch of every counter of a ``--pmc`` run, per kernel family.

``python -m paper_1603_03590_amd.profsum traffic <fetch_dir> <write_dir>
--kernel REGEX --copy-mib M --tile T --mode L`` prints the HBM traffic per launch of
the kernels matching REGEX, from two ``--pmc FETCH_SIZE`` / ``--pmc
WRITE_SIZE`` runs (``run_counter_collection.csv``, KiB per dispatch), each
counter scaled by what it reads for the run's plain device copy of M MiB
(the largest ``__amd_rocclr_copyBuffer`` dispatches), and a machine-readable
``traffic:`` line that bench.py matches against the kernel family, the
refinement tile, the launch mode and the hash of the kernel sources.

Every dispatch of the run is used; ``--after REGEX`` keeps only those after
the last dispatch whose kernel name matches (for a run whose autotuner
trials precede the timed launches; bench.py with ``--tunables`` has none).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/dis_kernels.hip", "csrc/dis_refine_tile.h", "csrc/dis_internal.h", "csrc/dis_lanes.h",
                  "csrc/dis_search_rows.h")
AFTER_DEFAULT = ""


def source_hash() -> str:
    """sha256 over the forward kernel sources (the traffic record's key)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def family(name: str) -> str:
    m = re.search(r"(k_\w+(<[^>]*>)?)", name)
    return m.group(1) if m else name.split("(")[0][:48]


def _after(rows, pattern):
    if not pattern:
        return rows
    idx = [i for i, r in enumerate(rows) if re.search(pattern, r["Kernel_Name"])]
    return rows[(max(idx) + 1) if idx else 0:]


def trace_table(d: str, after: str = AFTER_DEFAULT) -> str:
    rows = list(csv.DictReader(open(os.path.join(d, "run_kernel_trace.csv"))))
    rows = _after(rows, after)
    agg = {}
    for r in rows:
        k = family(r["Kernel_Name"])
        agg.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    tot = sum(sum(v) for v in agg.values())
    out = ["| Kernel | Calls | Total (us) | Average (us) | Median (us) | % |", "|:--|--:|--:|--:|--:|--:|"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| `{k}` | {len(v)} | {sum(v):.1f} | {sum(v) / len(v):.2f} | {statistics.median(v):.2f} | "
                   f"{100 * sum(v) / tot:.1f} |")
    return "\n".join(out)


def _counters(d):
    return list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))


def traffic_record(fetch_dir: str, write_dir: str, kernel: str, copy_mib: int, tile: int, mode: int,
                   after: str = AFTER_DEFAULT) -> tuple[str, dict]:
    F, Wr = _counters(fetch_dir), _counters(write_dir)
    expect = copy_mib * 1024.0   # KiB read and written by one copy

    def probe(rows):
        c = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        c = sorted(c)[-5:]
        return statistics.median(c) if c else float("nan")

    ff, fw = expect / probe(F), expect / probe(Wr)
    f_sel = [r for r in _after(F, after) if re.search(kernel, r["Kernel_Name"])]
    w_sel = [r for r in _after(Wr, after) if re.search(kernel, r["Kernel_Name"])]
    n = min(len(f_sel), len(w_sel))
    fetch = sum(float(r["Counter_Value"]) for r in f_sel[:n]) / n * ff * 1024.0
    write = sum(float(r["Counter_Value"]) for r in w_sel[:n]) / n * fw * 1024.0
    rec = dict(kernel=kernel, tile=tile, mode=mode, launches=n, fetch_bytes_per_launch=fetch,
               write_bytes_per_launch=write, bytes_per_launch=fetch + write, fetch_scale=ff, write_scale=fw,
               source_sha=source_hash())
    line = "traffic: " + " ".join(f"{k}={v:.6g}" if isinstance(v, float) else f"{k}={v}" for k, v in rec.items())
    return line, rec


def util_table(d: str, after: str = AFTER_DEFAULT) -> str:
    """Mean per dispatch of every collected counter, per kernel family
    (``--pmc`` run; derived metrics such as VALUBusy come computed)."""
    rows = _after(_counters(d), after)
    agg = {}
    for r in rows:
        k = family(r["Kernel_Name"])
        agg.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for v in agg.values() for c in v})
    out = ["| Kernel | dispatches | " + " | ".join(names) + " |", "|:--|--:|" + "--:|" * len(names)]
    for k, v in sorted(agg.items(), key=lambda kv: -len(next(iter(kv[1].values())))):
        n = max(len(x) for x in v.values())
        cells = [f"{statistics.mean(v[c]):.4g}" if c in v else "" for c in names]
        out.append(f"| `{k}` | {n} | " + " | ".join(cells) + " |")
    return "\n".join(out)


def read_traffic(path: str, tile: int | None = None, mode: int | None = None) -> dict | None:
    """The first ``traffic:`` record of a committed summary (with `tile` /
    `mode` given, the first one measured with them), or None."""
    try:
        for ln in open(path):
            if ln.startswith("traffic: "):
                rec = {}
                for kv in ln[len("traffic: "):].split():
                    k, v = kv.split("=", 1)
                    if k in ("tile", "mode", "launches"):
                        rec[k] = int(v)
                    elif k.endswith("_launch") or k.endswith("_scale"):
                        rec[k] = float(v)
                    else:
                        rec[k] = v
                if (tile is None or rec.get("tile") == tile) and (mode is None or rec.get("mode") == mode):
                    return rec
    except OSError:
        return None
    return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--after", default=AFTER_DEFAULT)
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--kernel", required=True)
    c.add_argument("--copy-mib", type=int, required=True)
    c.add_argument("--tile", type=int, required=True)
    c.add_argument("--mode", type=int, required=True, help="launch mode of the measured run")
    c.add_argument("--after", default=AFTER_DEFAULT)
    u = sub.add_parser("util")
    u.add_argument("dir")
    u.add_argument("--after", default=AFTER_DEFAULT)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_table(a.dir, a.after))
    elif a.cmd == "util":
        print(util_table(a.dir, a.after))
    else:
        line, rec = traffic_record(a.fetch_dir, a.write_dir, a.kernel, a.copy_mib, a.tile, a.mode, a.after)
        print(f"| counter | scale (copy probe) | KiB-scaled bytes per launch |\n|:--|--:|--:|\n"
              f"| FETCH_SIZE | {rec['fetch_scale']:.4f} | {rec['fetch_bytes_per_launch']:.0f} |\n"
              f"| WRITE_SIZE | {rec['write_scale']:.4f} | {rec['write_bytes_per_launch']:.0f} |\n")
        print(line)
    return 0


if __name__ == "__main__":
    sys.exit(main())
