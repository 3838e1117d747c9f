"""Summarise a rocprofv3 --stats kernel table into a short Markdown file.

    python -m paper_1512_02390_amd.profile_summary <run_kernel_stats.csv> <out.md> "<command>"
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


if __name__ == "__main__":
    main(*sys.argv[1:4])
