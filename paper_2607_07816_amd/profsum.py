"""Text summaries of rocprofv3 results (the SQLite `*_results.db` it writes).

    python -m paper_2607_07816_amd.profsum trace DB --command "..."
        per-kernel launch count and duration (kernel trace)
    python -m paper_2607_07816_amd.profsum traffic --fetch DB --write DB --copy-bytes B
                                           --kernel NAME --command "..."
        HBM bytes per launch of one kernel from FETCH_SIZE and WRITE_SIZE,
        each scaled by what the same counter reads for a device-to-device
        copy of B bytes in the same run
    python -m paper_2607_07816_amd.profsum counters DB [DB ...] --kernel PREFIX
                                           --command "..." [--command "..."]
        every collected counter per steady dispatch (and per wave) of the
        named kernels, one --pmc pass per database

Measurement tooling only: nothing here runs on the simulation path.
"""
from __future__ import annotations

import argparse
import collections
import glob
import hashlib
import os
import re
import sqlite3
import sys

_PKG = os.path.dirname(os.path.abspath(__file__))

SHORT_NAMES = ("k_radix_pass", "k_radix_count", "k_radix_hist", "k_radix_scan", "k_tile_hist", "k_tile_extract", "k_tile_emit",
               "k_tile_compact", "k_group_hist", "k_group_compact", "k_group_extract", "k_group_emit", "k_pick1",
               "k_side_hist", "k_side_extract", "k_final", "k_tile_kept", "k_tile_scan", "k_init_state",
               "k_set_n", "k_tile_sample", "k_fill_zero", "k_ctl_begin", "k_terms_out")


def short(name: str) -> str:
    """Readable kernel name: library kernels lose their template noise."""
    for key in SHORT_NAMES:
        if key in name:
            extra = ""
            if "float" in name:
                extra = "c64"
            elif "double" in name:
                extra = "c128"
            elif key == "k_radix_pass":  # templated on 64-bit words per amplitude
                w = re.search(r"k_radix_pass(?:<|ILi)(\d)", name)
                extra = {"1": "c64", "2": "c128"}.get(w.group(1), "") if w else ""
            m = re.search(r"Li(\d)E", name) if key != "k_radix_pass" else None
            if m and extra:
                extra += f",m={m.group(1)}"
            return key + (f"<{extra}>" if extra else "")
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0][:48] or name[:48]


def source_digest() -> str:
    """SHA-256 over every HIP source and header of the library: a profile
    taken at another digest describes other kernels."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(_PKG, "csrc", "*"))):
        if path.endswith((".hip", ".h")):
            h.update(os.path.basename(path).encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _db(path: str) -> sqlite3.Connection:
    if os.path.isdir(path):
        found = sorted(glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True))
        if not found:
            raise SystemExit(f"no *_results.db under {path}")
        path = found[0]
    return sqlite3.connect(path)


def kernel_rows(path: str, last: float = 0.5):
    """[(short name, calls, total_ns, avg_ns, min_ns, max_ns, steady_avg_ns)],
    largest total first. steady_avg is the mean over the last `last` fraction
    of each kernel's launches (the steady-state steps at the end of a run)."""
    cur = _db(path).cursor()
    durs = collections.defaultdict(list)
    for name, d in cur.execute("select name, duration from kernels order by start"):
        durs[short(name)].append(d)
    rows = []
    for k, d in durs.items():
        tail = d[int(len(d) * (1.0 - last)):] or d
        rows.append((k, len(d), sum(d), sum(d) / len(d), min(d), max(d), sum(tail) / len(tail)))
    return sorted(rows, key=lambda r: -r[2])


def counter_means(path: str, counter: str):
    """{short kernel name: (mean value per dispatch, dispatches)} for one
    counter over each kernel's largest-grid dispatches (the steady-state
    launches of the library's kernels; the calibration copy among the
    runtime's small blits)."""
    cur = _db(path).cursor()
    q = """select dispatch_id, kernel_name, grid_size, sum(value) from counters_collection
           where counter_name = ? group by dispatch_id"""
    rows = [(d, short(k), g, v) for d, k, g, v in cur.execute(q, (counter,))]
    best = {}
    for _, k, g, _ in rows:
        best[k] = max(best.get(k, 0), g)
    vals = collections.defaultdict(list)
    for _, k, g, v in rows:
        if g == best[k]:
            vals[k].append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}


def cmd_trace(args):
    rows = kernel_rows(args.db, args.last)
    tot = sum(r[2] for r in rows) or 1
    out = [f"# rocprofv3 kernel trace summary",
           f"# command: {args.command}",
           f"# library source digest: {source_digest()}",
           f"# steady_us: mean over the last {args.last:.0%} of each kernel's launches",
           f"{'kernel':32s} {'calls':>7s} {'total_us':>11s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} "
           f"{'steady_us':>10s} {'%':>6s}"]
    for k, n, t, a, lo, hi, st in rows:
        out.append(f"{k:32s} {n:7d} {t / 1e3:11.1f} {a / 1e3:9.2f} {lo / 1e3:9.2f} {hi / 1e3:9.2f} "
                   f"{st / 1e3:10.2f} {100 * t / tot:6.1f}")
    print("\n".join(out))


def _copy_entry(means):
    cands = [(k, v) for k, v in means.items() if "copy" in k.lower() and not k.startswith("k_")]
    if not cands:
        raise SystemExit("no copy kernel in the counter results (run bench.py with --copy-calibration)")
    return max(cands, key=lambda kv: kv[1][0])


def cmd_traffic(args):
    f = counter_means(args.fetch, "FETCH_SIZE")
    w = counter_means(args.write, "WRITE_SIZE")
    ck_f, (copy_f, _) = _copy_entry(f)
    ck_w, (copy_w, _) = _copy_entry(w)
    scale_f = args.copy_bytes / (copy_f * 1024.0)
    scale_w = args.copy_bytes / (copy_w * 1024.0)
    key = [k for k in f if k.startswith(args.kernel)]
    if not key:
        raise SystemExit(f"kernel {args.kernel} not in {sorted(f)}")
    k = max(key, key=lambda x: f[x][0])
    kf, nf = f[k]
    kw, nw = w.get(k, (0.0, 0))
    fetch_b = kf * 1024.0 * scale_f
    write_b = kw * 1024.0 * scale_w
    out = [f"# HBM traffic of {k} from rocprofv3 counters, copy-calibrated",
           f"# fetch command: {args.command_fetch or args.command}",
           f"# write command: {args.command_write or args.command}",
           f"# calibration: device-to-device copy of {args.copy_bytes} bytes ({ck_f}):",
           f"#   FETCH_SIZE {copy_f:.0f} KiB -> scale {scale_f:.4f}; WRITE_SIZE {copy_w:.0f} KiB -> scale {scale_w:.4f}",
           f"kernel: {args.kernel}",
           f"dispatches_fetch: {nf}",
           f"dispatches_write: {nw}",
           f"fetch_kib_per_launch_raw: {kf:.0f}",
           f"write_kib_per_launch_raw: {kw:.0f}",
           f"fetch_bytes_per_launch: {fetch_b:.0f}",
           f"write_bytes_per_launch: {write_b:.0f}",
           f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}",
           f"source_digest: {source_digest()}",
           "# all kernels (raw KiB per dispatch, FETCH_SIZE / WRITE_SIZE):"]
    for name in sorted(set(f) | set(w), key=lambda x: -f.get(x, (0, 0))[0]):
        out.append(f"#   {name:32s} {f.get(name, (0, 0))[0]:12.0f} {w.get(name, (0, 0))[0]:12.0f}")
    print("\n".join(out))


def cmd_counters(args):
    """Mean per steady dispatch of every counter in the given databases (one
    rocprofv3 --pmc pass each), for the kernels named by prefix; per wave
    too where SQ_WAVES was collected."""
    vals = collections.defaultdict(dict)
    for db in args.db:
        cur = _db(db).cursor()
        for (c,) in cur.execute("select distinct counter_name from counters_collection").fetchall():
            for k, (v, n) in counter_means(db, c).items():
                vals[k][c] = (v, n)
    kernels = [k for k in sorted(vals) if any(k.startswith(p) for p in args.kernel)]
    if not kernels:
        raise SystemExit(f"none of {args.kernel} in {sorted(vals)}")
    out = ["# rocprofv3 counters per dispatch (mean over each kernel's largest-grid dispatches)"]
    for i, cmd in enumerate(args.command):
        out.append(f"# command {i + 1}: {cmd}")
    out.append(f"# library source digest: {source_digest()}")
    for k in kernels:
        waves = vals[k].get("SQ_WAVES", (0.0, 0))[0]
        out.append(f"{k}  (dispatches: {max(n for _, n in vals[k].values())})")
        for c in sorted(vals[k]):
            v = vals[k][c][0]
            per_wave = f"{v / waves:14.1f} per wave" if waves and c != "SQ_WAVES" else ""
            out.append(f"  {c:28s} {v:16.4g} {per_wave}")
    print("\n".join(out))


def read_traffic(path: str):
    """Parse a traffic summary: {field: value} of its `name: value` lines."""
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--command", default="")
    t.add_argument("--last", type=float, default=0.5)
    c = sub.add_parser("traffic")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--command", default="")
    c.add_argument("--command-fetch", default="")
    c.add_argument("--command-write", default="")
    q = sub.add_parser("counters")
    q.add_argument("db", nargs="+")
    q.add_argument("--kernel", action="append", required=True, help="kernel name prefix (repeatable)")
    q.add_argument("--command", action="append", default=[], help="command of each pass (repeatable)")
    args = ap.parse_args(argv)
    {"trace": cmd_trace, "traffic": cmd_traffic, "counters": cmd_counters}[args.mode](args)


if __name__ == "__main__":
    sys.exit(main())
