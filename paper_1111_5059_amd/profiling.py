"""Summaries of rocprofv3 CSV output for the roofline report.

python -m paper_1111_5059_amd.profiling stats  <run_kernel_stats.csv> <kernel-substring> [command]
python -m paper_1111_5059_amd.profiling traffic <fetch_counter_collection.csv> <write_counter_collection.csv>
        <copy-bytes> <out.json>
python -m paper_1111_5059_amd.profiling counters <out.md> <counter_collection.csv> [more.csv ...]

``traffic`` converts FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of every hop and
fifth-dimension kernel variant in the run into HBM bytes per launch, each scaled by what the
same counter reads for a plain device copy of a known size (the last of the largest copy
kernels in the same run), and records the hash of the kernel sources so that a later kernel change
invalidates the figures.
"""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(f"none of {names} in {list(row)}")


def kernel_stats(path, substring):
    out = []
    for r in _rows(path):
        name = _col(r, "Name", "KernelName", "Kernel_Name")
        if substring in name:
            out.append({"name": name, "calls": int(_col(r, "Calls")),
                        "avg_ns": float(_col(r, "AverageNs", "Average_ns", "AverageNs ")),
                        "total_ns": float(_col(r, "TotalDurationNs", "TotalDuration_ns")),
                        "pct": float(_col(r, "Percentage"))})
    return out


def counter_per_dispatch(path, kernel_substring, counter):
    vals, grids = [], []
    for r in _rows(path):
        if _col(r, "Counter_Name") != counter:
            continue
        if kernel_substring in _col(r, "Kernel_Name"):
            vals.append(float(_col(r, "Counter_Value")))
            grids.append(int(_col(r, "Grid_Size")))
    return vals, grids


FAMILIES = ("hop_kernel<", "hop_eo5_kernel<", "hop_ilv_kernel<", "hop_batch_kernel<", "fifth_kernel<", "force_kernel<")


def short_name(full):
    """template instance of a hop / fifth-dimension kernel, without namespace and arguments"""
    for fam in FAMILIES:
        i = full.find(fam)
        if i < 0:
            continue
        depth, j = 0, i + len(fam) - 1
        while j < len(full):
            depth += {"<": 1, ">": -1}.get(full[j], 0)
            if depth == 0:
                return full[i:j + 1]
            j += 1
    return None


def per_kernel(path, counter):
    out = {}
    for r in _rows(path):
        if _col(r, "Counter_Name") != counter:
            continue
        k = short_name(_col(r, "Kernel_Name"))
        if k is not None:
            out.setdefault(k, []).append(float(_col(r, "Counter_Value")))
    return out


def copy_counter(path, counter):
    """counter of the calibration copy: the last dispatch of the largest-grid device copy kernel
    (``bench.py --only-hop`` ends with a 1 GiB device copy; solver copies of the same grid size
    may come earlier in the run)"""
    best = None
    for r in _rows(path):
        if _col(r, "Counter_Name") != counter:
            continue
        name = _col(r, "Kernel_Name")
        if "copy" in name.lower():
            g, d = int(_col(r, "Grid_Size")), int(_col(r, "Dispatch_Id"))
            if best is None or (g, d) > (best[0], best[3]):
                best = (g, float(_col(r, "Counter_Value")), name, d)
    return best


def counter_table(paths):
    """{kernel instance: {counter: mean per dispatch}} over one or more --pmc runs (each run may
    hold other counters of the same kernels)."""
    acc = {}
    for path in paths:
        for r in _rows(path):
            k = short_name(_col(r, "Kernel_Name"))
            if k is None:
                continue
            c = _col(r, "Counter_Name")
            acc.setdefault(k, {}).setdefault(c, []).append(float(_col(r, "Counter_Value")))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


def counters_markdown(table):
    cols = sorted({c for cs in table.values() for c in cs})
    lines = ["| kernel | " + " | ".join(cols) + " |", "|---|" + "---|" * len(cols)]
    for k in sorted(table):
        lines.append(f"| `{k}` | " + " | ".join(f"{table[k].get(c, float('nan')):.4g}" for c in cols) + " |")
    return "\n".join(lines) + "\n"


def main(argv):
    if argv[0] == "stats":
        for k in kernel_stats(argv[1], argv[2]):
            print(json.dumps(k))
        return
    if argv[0] == "traffic":
        fetch_csv, write_csv, copy_bytes, out = argv[1], argv[2], int(argv[3]), argv[4]
        f = per_kernel(fetch_csv, "FETCH_SIZE")
        w = per_kernel(write_csv, "WRITE_SIZE")
        cf = copy_counter(fetch_csv, "FETCH_SIZE")
        cw = copy_counter(write_csv, "WRITE_SIZE")
        fscale = copy_bytes / (cf[1] * 1024.0)
        wscale = copy_bytes / (cw[1] * 1024.0)
        kernels = {}
        for k in sorted(set(f) & set(w)):
            fetch = sum(f[k]) / len(f[k]) * 1024.0 * fscale
            write = sum(w[k]) / len(w[k]) * 1024.0 * wscale
            kernels[k] = {"dispatches": len(f[k]), "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
                          "hbm_bytes_per_launch": fetch + write}
        sys.path.insert(0, ROOT)
        import bench
        d = {"copy_kernel": cf[2][:120], "copy_bytes": copy_bytes, "fetch_scale": fscale, "write_scale": wscale,
             "kernel_source_sha256_16": bench.kernel_source_hash(), "kernels": kernels}
        with open(out, "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d))
        return
    if argv[0] == "counters":
        table = counter_table(argv[2:])
        with open(argv[1], "w") as fh:
            fh.write(counters_markdown(table))
        print(json.dumps(table))
        return
    raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
