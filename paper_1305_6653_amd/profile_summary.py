"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as a short text table.

    python -m paper_1305_6653_amd.profile_summary <results.db> [--title T] [--command C]
"""
import argparse
import sqlite3


def summarise(db: str, top: int = 25):
    c = sqlite3.connect(db)
    rows = list(c.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration), "
        "max(vgpr_count), max(accum_vgpr_count), max(lds_size), max(grid_x*grid_y*grid_z), "
        "max(workgroup_x*workgroup_y*workgroup_z) from kernels group by name "
        "order by sum(duration) desc"))
    total = sum(r[2] for r in rows) or 1.0
    return rows[:top], total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="")
    a = ap.parse_args()
    rows, total = summarise(a.db)
    if a.title:
        print(a.title)
    if a.command:
        print(f"command: {a.command}")
    print(f"{'kernel':58s} {'calls':>6s} {'total_us':>11s} {'avg_us':>10s} {'min_us':>9s} "
          f"{'max_us':>9s} {'pct':>6s} {'vgpr':>5s} {'agpr':>5s} {'lds':>7s} {'grid':>10s} {'wg':>5s}")
    for name, n, tot, avg, mn, mx, vg, ag, lds, grid, wg in rows:
        short = name.split("(")[0].replace("void ", "")[:58]
        print(f"{short:58s} {n:6d} {tot / 1e3:11.1f} {avg / 1e3:10.2f} {mn / 1e3:9.2f} {mx / 1e3:9.2f} "
              f"{100 * tot / total:6.2f} {vg:5d} {ag:5d} {lds:7d} {grid:10d} {wg:5d}")


if __name__ == "__main__":
    main()
