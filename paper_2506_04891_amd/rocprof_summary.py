"""Short text summaries of rocprofv3 output databases (rocpd SQLite files).

    python -m paper_2506_04891_amd.rocprof_summary trace RUN_results.db --command "..."
        per-kernel calls, total and average duration (kernel trace + stats run)

    python -m paper_2506_04891_amd.rocprof_summary counters RUN_results.db --command "..."
        per-kernel averages of every counter collected (one --pmc run)

    python -m paper_2506_04891_amd.rocprof_summary traffic --fetch F.db --write W.db \
        --kernel SUBSTR --copy-kernel SUBSTR --copy-bytes N --command-fetch "..." --command-write "..."
        HBM bytes per launch of the kernels matching SUBSTR (pooled) from FETCH_SIZE / WRITE_SIZE counter
        runs, each scaled by what the same counter reads for a plain streaming
        kernel that moves a known number of bytes in the same run

Both print `key: value` text meant to be kept next to the numbers it backs.
"""
import argparse
import collections
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def sources_sha256():
    """Hash of the native sources (kernels, planner, ABI): a traffic figure is
    only valid for the code it was measured on."""
    h = hashlib.sha256()
    root = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(root)):
        if name.endswith((".hip", ".h", ".cpp", ".inc")):
            with open(os.path.join(root, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    hdr = os.path.join(os.path.dirname(HERE), "include", "tqsim.h")
    with open(hdr, "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def _kernels(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration, lds_size, vgpr_count, accum_vgpr_count, sgpr_count, "
                       "scratch_size, grid_x, workgroup_x from kernels").fetchall()
    con.close()
    return rows


def trace_summary(db, command):
    stats = collections.OrderedDict()
    for name, dur, lds, vgpr, agpr, sgpr, scr, gx, wx in _kernels(db):
        s = stats.setdefault(name, {"calls": 0, "ns": [], "meta": (lds, vgpr, agpr, sgpr, scr, wx)})
        s["calls"] += 1
        s["ns"].append(dur)
    total = sum(sum(s["ns"]) for s in stats.values())
    out = [f"command: {command}", f"database: {os.path.basename(db)}",
           "columns: calls | total_ms | avg_us | min_us | max_us | pct | lds_B vgpr agpr sgpr scratch_B wg | kernel"]
    for name, s in sorted(stats.items(), key=lambda kv: -sum(kv[1]["ns"])):
        ns = s["ns"]
        lds, vgpr, agpr, sgpr, scr, wx = s["meta"]
        out.append(f"{s['calls']:6d} | {sum(ns) / 1e6:10.3f} | {sum(ns) / len(ns) / 1e3:9.2f} | "
                   f"{min(ns) / 1e3:9.2f} | {max(ns) / 1e3:9.2f} | {100.0 * sum(ns) / max(total, 1):5.1f} | "
                   f"{lds} {vgpr} {agpr} {sgpr} {scr} {wx} | {name}")
    return "\n".join(out)


def _counter(db, counter):
    """Per-kernel list of per-dispatch counter values (summed over the
    counter's instances)."""
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection").fetchall()
    con.close()
    per = collections.defaultdict(float)
    names = {}
    for d, k, c, v in rows:
        if c == counter:
            per[d] += v
            names[d] = k
    out = collections.defaultdict(list)
    for d, v in per.items():
        out[names[d]].append(v)
    return out


def counters_summary(db, command):
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection").fetchall()
    con.close()
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for d, k, c, v in rows:
        per[d][c] += v
        names[d] = k
    agg = collections.OrderedDict()
    for d, cs in per.items():
        a = agg.setdefault(names[d], collections.defaultdict(list))
        for c, v in cs.items():
            a[c].append(v)
    out = [f"command: {command}", f"database: {os.path.basename(db)}",
           "per-dispatch averages, summed over counter instances"]
    for k, cs in agg.items():
        n = len(next(iter(cs.values())))
        vals = " ".join(f"{c}={sum(v) / len(v):.4g}" for c, v in sorted(cs.items()))
        out.append(f"{k} | dispatches={n} | {vals}")
    return "\n".join(out)


def _pick(per_kernel, sub):
    keys = [k for k in per_kernel if sub in k]
    if len(keys) != 1:
        raise SystemExit(f"kernel substring {sub!r} matches {keys}")
    return keys[0], per_kernel[keys[0]]


def _pick_all(per_kernel, sub):
    """Every kernel whose name contains `sub` (e.g. all template variants of
    one pass kind), with their dispatches pooled."""
    keys = sorted(k for k in per_kernel if sub in k)
    if not keys:
        raise SystemExit(f"kernel substring {sub!r} matches nothing")
    return " + ".join(keys), [v for k in keys for v in per_kernel[k]]


def traffic_summary(a):
    fetch = _counter(a.fetch, "FETCH_SIZE")
    write = _counter(a.write, "WRITE_SIZE")
    ck, cf = _pick(fetch, a.copy_kernel)
    _, cw = _pick(write, a.copy_kernel)
    kk, kf = _pick_all(fetch, a.kernel)
    _, kw = _pick_all(write, a.kernel)
    kib = a.copy_bytes / 1024.0
    cf_avg, cw_avg = sum(cf) / len(cf), sum(cw) / len(cw)
    f_fac, w_fac = kib / cf_avg, kib / cw_avg
    kf_avg, kw_avg = sum(kf) / len(kf), sum(kw) / len(kw)
    traffic = (kf_avg * f_fac + kw_avg * w_fac) * 1024.0
    lines = [
        f"command_fetch: {a.command_fetch}",
        f"command_write: {a.command_write}",
        f"kernel: {kk}",
        f"profile_kind: {a.profile_kind}",
        f"copy_kernel: {ck}",
        f"copy_bytes_read_and_written_per_dispatch: {a.copy_bytes}",
        f"copy_fetch_kib_per_dispatch: {cf_avg:.1f}",
        f"copy_write_kib_per_dispatch: {cw_avg:.1f}",
        f"fetch_factor: {f_fac:.4f}",
        f"write_factor: {w_fac:.4f}",
        f"kernel_dispatches: {len(kf)}",
        f"kernel_fetch_kib_per_dispatch_raw: {kf_avg:.1f}",
        f"kernel_write_kib_per_dispatch_raw: {kw_avg:.1f}",
        f"traffic_bytes_per_launch: {traffic:.0f}",
        f"sources_sha256: {a.sha or sources_sha256()}",
    ]
    return "\n".join(lines)


def read_traffic(path, profile_kind):
    """Traffic bytes per launch from a summary written by `traffic`, or None
    when the file is absent, names another kernel, or was taken on other
    sources than the ones built now."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("profile_kind") != profile_kind or kv.get("sources_sha256") != sources_sha256():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main(argv=None):
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--command", required=True)
    q = sub.add_parser("counters")
    q.add_argument("db")
    q.add_argument("--command", required=True)
    r = sub.add_parser("traffic")
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--kernel", required=True)
    r.add_argument("--profile-kind", required=True)
    r.add_argument("--copy-kernel", required=True)
    r.add_argument("--copy-bytes", type=float, required=True)
    r.add_argument("--command-fetch", required=True)
    r.add_argument("--command-write", required=True)
    r.add_argument("--sha", default=None)
    a = p.parse_args(argv)
    if a.cmd == "trace":
        print(trace_summary(a.db, a.command))
    elif a.cmd == "counters":
        print(counters_summary(a.db, a.command))
    else:
        print(traffic_summary(a))


if __name__ == "__main__":
    sys.exit(main())
