"""Summaries of rocprofv3 output as short Markdown / JSON files.

    python -m paper_1512_02390_amd.profile_summary <run_kernel_stats.csv> <out.md> "<command>"
    python -m paper_1512_02390_amd.profile_summary traffic <fetch.csv> <write.csv> \
        <copy_fetch.csv> <copy_write.csv> <copy_bytes> <kernel substring> <key> \
        <source hash> <out.json> <out.md> "<cmd1;;cmd2;;...>"
"""
import csv
import sys


def main(src, dst, command):
    rows = list(csv.DictReader(open(src)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
             "| share | calls | avg (us) | total (us) | kernel |", "|---:|---:|---:|---:|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"].replace("sem::(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| {float(r['TotalDurationNs']) / tot * 100:.1f}% | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                     f"`{name}` |")
    lines.append("")
    lines.append(f"Total kernel time: {tot / 1e3:.1f} us")
    open(dst, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__" and sys.argv[1:2] != ["traffic"]:
    main(*sys.argv[1:4])


def _per_dispatch(csv_path, counter):
    """{kernel name: [counter value per dispatch]} from a rocprofv3 --pmc CSV."""
    out = {}
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def traffic(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, copy_bytes, kernel, key,
            source_hash, dst_json, dst_md, commands):
    """HBM bytes per launch of `kernel` from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by the factor that maps the same counter of a plain
    copy of `copy_bytes` bytes onto the bytes it must move."""
    import json
    import os
    copy_bytes = float(copy_bytes)

    def copy_factor(path, counter):
        vals = [v for vs in _per_dispatch(path, counter).values() for v in vs]
        big = max(vals)   # the large copy dwarfs every other dispatch
        return copy_bytes / (big * 1024.0), big

    ff, fraw = copy_factor(cal_fetch_csv, "FETCH_SIZE")
    fw, wraw = copy_factor(cal_write_csv, "WRITE_SIZE")

    def mean_for(path, counter):
        d = _per_dispatch(path, counter)
        vals = [v for name, vs in d.items() if kernel in name for v in vs]
        return sum(vals) / len(vals), len(vals)

    fetch_kib, nf = mean_for(fetch_csv, "FETCH_SIZE")
    write_kib, nw = mean_for(write_csv, "WRITE_SIZE")
    total = fetch_kib * 1024.0 * ff + write_kib * 1024.0 * fw
    rec = {}
    if os.path.exists(dst_json):
        rec = json.load(open(dst_json))
    if rec.get("source_hash") != source_hash:
        rec = {"source_hash": source_hash, "per_launch": {}, "detail": {}}
    rec["per_launch"][key] = total
    rec["detail"][key] = {"kernel": kernel, "fetch_kib": fetch_kib, "write_kib": write_kib,
                          "dispatches": [nf, nw], "copy_factor_fetch": ff,
                          "copy_factor_write": fw, "copy_fetch_kib": fraw,
                          "copy_write_kib": wraw, "copy_bytes": copy_bytes}
    json.dump(rec, open(dst_json, "w"), indent=1)
    lines = ["# HBM traffic of `%s` (%s)" % (kernel, key), "", "Commands:", "", "```"] + \
            commands.split(";;") + ["```", "",
            "| quantity | value |", "|---|---|",
            f"| FETCH_SIZE per dispatch | {fetch_kib:.1f} KiB ({nf} dispatches) |",
            f"| WRITE_SIZE per dispatch | {write_kib:.1f} KiB ({nw} dispatches) |",
            f"| copy of {copy_bytes / 2**20:.0f} MiB: FETCH_SIZE / WRITE_SIZE | "
            f"{fraw:.0f} / {wraw:.0f} KiB |",
            f"| scale factors (bytes per counted byte) | fetch {ff:.3f}, write {fw:.3f} |",
            f"| HBM bytes per launch | {total / 1e6:.3f} MB |", ""]
    open(dst_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "traffic":
    traffic(*sys.argv[2:14])
