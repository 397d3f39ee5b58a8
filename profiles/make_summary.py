"""Turn a rocprofv3 --kernel-trace --stats CSV into the short text summary kept in profiles/.

usage: python profiles/make_summary.py <kernel_stats.csv> <title> <command> > profiles/<name>.md
"""
import csv
import sys


def main():
    path, title, cmd = sys.argv[1], sys.argv[2], sys.argv[3]
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    print("# %s\n" % title)
    print("Command (run from the repository root on the GPU box):\n\n    %s\n" % cmd)
    print("Total kernel time %.1f ms over %d kernels.\n" % (tot / 1e6, len(rows)))
    print("| kernel | calls | total ms | avg us | share |")
    print("|---|---:|---:|---:|---:|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:20]:
        name = r["Name"].split("(")[0].replace("gck::", "").replace("void ", "")
        print("| %s | %s | %.2f | %.2f | %.1f%% |" % (name, r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                      float(r["AverageNs"]) / 1e3, float(r["Percentage"])))


if __name__ == "__main__":
    main()
