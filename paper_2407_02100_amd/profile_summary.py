"""Summarise a rocprofv3 kernel trace (rocpd SQLite output) per kernel and grid.

Usage: python -m paper_2407_02100_amd.profile_summary RESULTS_DB [--top N] [--grids G]

Prints, per kernel name, the number of dispatches, total and average
duration, and the same split by launch grid (which separates the levels of
the multigrid hierarchy for kernels shared by all levels).
"""
from __future__ import annotations

import argparse
import sqlite3
from collections import defaultdict


def summarise(db_path: str, top: int = 12, grids_per_kernel: int = 6) -> str:
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, duration, grid_x, grid_y, grid_z, workgroup_x from kernels").fetchall()
    by_name = defaultdict(list)
    by_grid = defaultdict(list)
    for name, dur, gx, gy, gz, wx in rows:
        by_name[name].append(dur)
        by_grid[(name, gx, gy, gz, wx)].append(dur)
    total = sum(sum(v) for v in by_name.values())
    lines = [f"# {len(rows)} dispatches, {total / 1e6:.3f} ms of kernel time (durations in ns below -> us)",
             f"{'kernel':<90} {'calls':>6} {'total_us':>11} {'avg_us':>10} {'pct':>6}"]
    names = sorted(by_name, key=lambda n: -sum(by_name[n]))[:top]
    for n in names:
        d = by_name[n]
        lines.append(f"{n[:90]:<90} {len(d):>6} {sum(d) / 1e3:>11.1f} {sum(d) / len(d) / 1e3:>10.2f} "
                     f"{100 * sum(d) / total:>6.2f}")
    lines.append("")
    lines.append("# split by launch grid (grid_x, grid_y, grid_z in work-items; workgroup size)")
    for n in names[:4]:
        grids = sorted((k for k in by_grid if k[0] == n), key=lambda k: -(k[1] * k[2] * k[3]))
        for k in grids[:grids_per_kernel]:
            d = by_grid[k]
            lines.append(f"{n[:60]:<60} grid=({k[1]},{k[2]},{k[3]}) wg={k[4]} calls={len(d)} "
                         f"avg_us={sum(d) / len(d) / 1e3:.2f}")
    return "\n".join(lines)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--grids", type=int, default=6, help="launch grids listed per kernel (largest first)")
    a = ap.parse_args()
    print(summarise(a.db, a.top, a.grids))
