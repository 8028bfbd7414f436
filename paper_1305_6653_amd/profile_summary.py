"""Summaries of rocprofv3 output as short text tables.

Kernel trace (rocpd SQLite database written by ``rocprofv3 --kernel-trace --stats``):

    python -m paper_1305_6653_amd.profile_summary trace <results.db> [--title T] [--command C]

Hardware counters (CSV written by ``rocprofv3 --pmc FETCH_SIZE -f csv`` and, in a second run,
``--pmc WRITE_SIZE``): average KiB per dispatch per kernel, and the same figures scaled to bytes
by a reference copy dispatch of known size (the largest dispatch whose name matches
``--copy-kernel``, which read and wrote ``--copy-bytes`` bytes):

    python -m paper_1305_6653_amd.profile_summary pmc <fetch.csv> <write.csv> --copy-bytes N \
        [--split NAME_SUBSTRING:KiB ...]

Any counters (e.g. SQ_INSTS_VALU_MFMA_MOPS_F64, SQ_VALU_MFMA_BUSY_CYCLES): per-kernel averages:

    python -m paper_1305_6653_amd.profile_summary counters <counter_collection.csv> [--key C]
"""
import argparse
import csv
import re
import sqlite3
from collections import defaultdict


def summarise(db: str, top: int = 25, splits=()):
    """Per-kernel rows; splits = ["name_substring:us", ...] report a kernel's dispatches shorter
    and longer than us apart (e.g. one block-solve kernel applying full LU factors or U only)."""
    c = sqlite3.connect(db)
    rules = [(sub, float(us)) for sub, us in (x.rsplit(":", 1) for x in splits)]
    tag = "name"
    for sub, us in rules:
        tag = (f"case when instr(name, '{sub}') > 0 then name || case when duration >= {us * 1e3} "
               f"then ' [>={us:g} us]' else ' [<{us:g} us]' end else {tag} end")
    rows = list(c.execute(
        f"select {tag} as nm, count(*), sum(duration), avg(duration), min(duration), max(duration), "
        "max(vgpr_count), max(accum_vgpr_count), max(lds_size), max(grid_x*grid_y*grid_z), "
        "max(workgroup_x*workgroup_y*workgroup_z), min(name) from kernels group by nm "
        "order by sum(duration) desc"))
    total = sum(r[2] for r in rows) or 1.0
    return rows[:top], total


def short_name(name: str) -> str:
    """Kernel name without its argument list; a split tag (" [...]") is kept."""
    if "(" not in name:
        return name.replace("void ", "").strip()
    tail = name[name.rindex(" ["):] if name.endswith("]") and " [" in name else ""
    return name.split("(")[0].replace("void ", "").strip() + tail


def active_stats(db: str, name: str, frac: float = 0.05, lo_ns: float = 0.0, hi_ns: float = 1e30):
    """(count, average ns) over the dispatches of `name` (with durations in [lo_ns, hi_ns)) that
    last at least frac x the median: launches whose workgroups all found their instance gated
    off (nothing to do) are left out."""
    c = sqlite3.connect(db)
    d = sorted(r[0] for r in c.execute("select duration from kernels where name = ?", (name,))
               if lo_ns <= r[0] < hi_ns)
    if not d:
        return 0, 0.0
    cut = frac * d[len(d) // 2]
    act = [x for x in d if x >= cut]
    return len(act), (sum(act) / len(act) if act else 0.0)


def trace_main(a):
    rows, total = summarise(a.db, splits=a.split or [])
    if a.title:
        print(a.title)
    if a.command:
        print(f"command: {a.command}")
    print("act_calls / act_avg_us: dispatches lasting at least 5% of the kernel's median (the others "
          "found every instance gated off)")
    print(f"{'kernel':50s} {'calls':>6s} {'total_us':>11s} {'avg_us':>10s} {'min_us':>9s} "
          f"{'max_us':>9s} {'act_calls':>9s} {'act_avg_us':>10s} {'pct':>6s} {'vgpr':>5s} {'lds':>7s} {'grid':>10s} {'wg':>5s}")
    for name, n, tot, avg, mn, mx, vg, ag, lds, grid, wg, raw in rows:
        short = short_name(name)[-50:] if name.endswith("]") else short_name(name)[:50]
        lo, hi = 0.0, 1e30
        if name.endswith(" us]"):  # a split row: "[>=X us]" or "[<X us]"
            tag = name[name.rindex("[") + 1:-4]
            if tag.startswith(">="):
                lo = float(tag[2:]) * 1e3
            else:
                hi = float(tag[1:]) * 1e3
        na, aa = active_stats(a.db, raw, lo_ns=lo, hi_ns=hi)
        print(f"{short:50s} {n:6d} {tot / 1e3:11.1f} {avg / 1e3:10.2f} {mn / 1e3:9.2f} {mx / 1e3:9.2f} "
              f"{na:9d} {aa / 1e3:10.2f} {100 * tot / total:6.2f} {vg:5d} {lds:7d} {grid:10d} {wg:5d}")


def _col(header, *keys):
    for k in keys:
        for i, h in enumerate(header):
            if h.strip().lower() == k.lower():
                return i
    raise KeyError(f"none of {keys} in CSV header {header}")


def read_counter(path: str, counter: str):
    """{dispatch id: (kernel name, value)} for one counter of a counter-collection CSV."""
    out = {}
    with open(path, newline="") as fh:
        rd = csv.reader(fh)
        header = next(rd)
        ik = _col(header, "Kernel_Name", "Kernel-Name", "KernelName")
        ic = _col(header, "Counter_Name", "Counter-Name")
        iv = _col(header, "Counter_Value", "Counter-Value")
        idd = _col(header, "Dispatch_Id", "Dispatch-Id", "Correlation_Id")
        for row in rd:
            if row[ic].strip() != counter:
                continue
            d = row[idd]
            name, v = row[ik], float(row[iv])
            prev = out.get(d)
            out[d] = (name, v + (prev[1] if prev else 0.0))
    return out


def pair_by_order(fetch, write):
    """The two counter runs are separate executions of the same program: the k-th dispatch of a
    kernel in one matches the k-th dispatch of that kernel in the other (dispatch ids can shift
    when other kernels' launch counts differ).  Returns [(name, fetch, write or None)]."""
    fl, wl = defaultdict(list), defaultdict(list)
    for d in sorted(fetch, key=lambda x: int(x) if str(x).isdigit() else x):
        fl[fetch[d][0]].append(fetch[d][1])
    for d in sorted(write, key=lambda x: int(x) if str(x).isdigit() else x):
        wl[write[d][0]].append(write[d][1])
    out = []
    for n, fv in fl.items():
        wv = wl.get(n, [])
        for k, v in enumerate(fv):
            out.append((n, v, wv[k] if k < len(wv) else None))
    return out


def traffic_per_dispatch(pairs, splits=(), frac: float = 0.05):
    """{kernel: [n, sum_fetch, n_write, sum_write]} over the dispatches whose FETCH_SIZE is at
    least frac x the kernel's median (gated-off launches, which read only their control data,
    are left out).  splits = ["name_substring:KiB", ...] report a kernel's dispatches fetching
    at least KiB apart from the others (e.g. one block-solve kernel applying full LU factors or
    U only)."""
    rules = [(sub, float(kib)) for sub, kib in (x.rsplit(":", 1) for x in splits)]

    def tagged(n, v):
        t = short_name(n)
        for sub, kib in rules:
            if sub in n:
                t += f" [{'>=' if v >= kib else '<'}{kib:g} KiB]"
        return t
    by_name = defaultdict(list)
    for n, v, _ in pairs:
        by_name[tagged(n, v)].append(v)
    cut = {k: frac * sorted(v)[len(v) // 2] for k, v in by_name.items()}
    agg = defaultdict(lambda: [0, 0.0, 0, 0.0])
    for n, v, w in pairs:
        t = tagged(n, v)
        if v < cut[t]:
            continue
        e = agg[t]
        e[0] += 1
        e[1] += v
        if w is not None:
            e[2] += 1
            e[3] += w
    return agg


def pmc_main(a):
    fetch = read_counter(a.fetch_csv, "FETCH_SIZE")
    write = read_counter(a.write_csv, "WRITE_SIZE")
    pat = re.compile(a.copy_kernel)

    def largest_copy(tab):
        cands = [v for (n, v) in tab.values() if pat.search(n)]
        if not cands:
            raise SystemExit(f"no dispatch matches {a.copy_kernel!r}")
        return max(cands)

    kib = a.copy_bytes / 1024.0
    f_scale = kib / largest_copy(fetch)
    w_scale = kib / largest_copy(write)
    agg = traffic_per_dispatch(pair_by_order(fetch, write), a.split or [])
    if a.title:
        print(a.title)
    for c in a.command or []:
        print(f"command: {c}")
    print(f"reference copy: {a.copy_bytes} bytes read and written; FETCH_SIZE scale {f_scale:.4f}, "
          f"WRITE_SIZE scale {w_scale:.4f} (bytes = KiB counter x 1024 x scale)")
    print(f"{'kernel':44s} {'disp':>6s} {'FETCH_KiB/disp':>15s} {'WRITE_KiB/disp':>15s} "
          f"{'read_MB/disp':>13s} {'write_MB/disp':>13s} {'HBM_MB/disp':>12s}")
    rows = sorted(agg.items(), key=lambda kv: -(kv[1][1] + kv[1][3]))
    for name, (nf, sf, nw, sw) in rows[:a.top]:
        fa = sf / nf if nf else 0.0
        wa = sw / nw if nw else 0.0
        rb = fa * 1024 * f_scale / 1e6
        wb = wa * 1024 * w_scale / 1e6
        print(f"{name[:44]:44s} {max(nf, nw):6d} {fa:15.1f} {wa:15.1f} {rb:13.3f} {wb:13.3f} {rb + wb:12.3f}")


def counters_main(a):
    """Per kernel: dispatches and the average of every counter in the CSV (dispatches whose key
    counter is below 5% of the kernel's median are left out, as gated-off launches)."""
    tabs = {}
    with open(a.csv, newline="") as fh:
        rd = csv.reader(fh)
        header = next(rd)
        ik = _col(header, "Kernel_Name", "Kernel-Name", "KernelName")
        ic = _col(header, "Counter_Name", "Counter-Name")
        iv = _col(header, "Counter_Value", "Counter-Value")
        idd = _col(header, "Dispatch_Id", "Dispatch-Id", "Correlation_Id")
        for row in rd:
            d, c = row[idd], row[ic].strip()
            e = tabs.setdefault(d, [row[ik], {}])
            e[1][c] = e[1].get(c, 0.0) + float(row[iv])
    names = sorted({c for _, cs in tabs.values() for c in cs})
    first = names[0] if not a.key else a.key
    by = defaultdict(list)
    for n, cs in tabs.values():
        by[short_name(n)].append(cs)
    if a.title:
        print(a.title)
    for c in a.command or []:
        print(f"command: {c}")
    util = a.simds > 0 and "SQ_VALU_MFMA_BUSY_CYCLES" in names and "GRBM_GUI_ACTIVE" in names
    extra = ["mfma_busy_frac", "mfma_flops/disp"] if util else []
    if util:
        print(f"mfma_busy_frac = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {a.xcds} x {a.simds} SIMDs) "
              "(the busy cycles summed over every SIMD, the active cycles over the XCDs); "
              "mfma_flops/disp = (SQ_INSTS_VALU_MFMA_MOPS_F64 + _F32) x 512")
    print(f"{'kernel':44s} {'disp':>6s} " + " ".join(f"{c:>28s}" for c in names + extra))
    rows = []
    for n, lst in by.items():
        med = sorted(x.get(first, 0.0) for x in lst)[len(lst) // 2]
        act = [x for x in lst if x.get(first, 0.0) >= 0.05 * med] or lst
        avg = {c: sum(x.get(c, 0.0) for x in act) / len(act) for c in names}
        rows.append((n, len(act), avg))
    rows.sort(key=lambda r: -r[2].get(first, 0.0) * r[1])
    for n, k, avg in rows[:a.top]:
        vals = [avg[c] for c in names]
        if util:
            act = avg["GRBM_GUI_ACTIVE"] / a.xcds * a.simds
            vals.append(avg["SQ_VALU_MFMA_BUSY_CYCLES"] / act if act > 0 else 0.0)
            vals.append(512.0 * (avg.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) + avg.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)))
        print(f"{n[:44]:44s} {k:6d} " + " ".join(f"{v:28.4g}" for v in vals))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--title", default="")
    t.add_argument("--command", default="")
    t.add_argument("--split", action="append",
                   help="NAME_SUBSTRING:us: report a kernel's dispatches shorter and longer than us apart")
    p = sub.add_parser("pmc")
    p.add_argument("fetch_csv")
    p.add_argument("write_csv")
    p.add_argument("--copy-bytes", type=float, required=True)
    p.add_argument("--copy-kernel", default="copyBuffer")
    p.add_argument("--title", default="")
    p.add_argument("--command", action="append")
    p.add_argument("--top", type=int, default=25)
    p.add_argument("--split", action="append",
                   help="NAME_SUBSTRING:KiB: report a kernel's dispatches below and above KiB apart")
    g = sub.add_parser("counters")
    g.add_argument("csv")
    g.add_argument("--key", default="", help="counter that orders the rows and sets the gated-off cut")
    g.add_argument("--title", default="")
    g.add_argument("--command", action="append")
    g.add_argument("--top", type=int, default=25)
    g.add_argument("--xcds", type=int, default=8, help="XCDs whose GRBM_GUI_ACTIVE counts are summed")
    g.add_argument("--simds", type=int, default=0, help="SIMDs of the device (1024 on MI355X): adds the MFMA busy fraction")
    a = ap.parse_args()
    {"trace": trace_main, "pmc": pmc_main, "counters": counters_main}[a.mode](a)


if __name__ == "__main__":
    main()
