"""Turn rocprofv3 CSV output into the short summaries kept with the library.

* ``trace``: ``--kernel-trace --stats`` output -> Markdown table of kernels.
* ``traffic``: two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of
  ``bench.py --copy-calibration MIB`` -> HBM bytes per launch of the product
  kernel.  Each counter is scaled by what it reads for the calibration copy
  (an elementwise kernel that reads and writes MIB MiB once), so the figures
  are bytes, whatever unit and coverage the counter has on this GPU.  The
  result records the hash of the kernel source it was taken on; bench.py
  only reports it while that source is unchanged.

Usage::

    python -m paper_2303_04353_amd.profiling trace DIR/run_kernel_stats.csv [--cmd "..."]
    python -m paper_2303_04353_amd.profiling traffic FETCH.csv WRITE.csv --copy-mib 1024 \\
        --m 8192 --n 8192 --k 8192 --out profiles/<name>.json
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# the headline form of the product kernel: no flags, global Sigma and T, 64 x 64 tiles
PRODUCT_KERNEL = "cascade_kernel<false, false, Shape<64, 64> >"
PRODUCT_SOURCE = os.path.join(HERE, "csrc", "cascade.hip")


def is_product_kernel(name: str) -> bool:
    """True for the headline product kernel's name as rocprofv3 prints it
    (namespaces of the template arguments dropped)."""
    plain = name.replace("(anonymous namespace)::", "").replace("ddk::", "")
    return PRODUCT_KERNEL in plain


def source_hash(path: str = PRODUCT_SOURCE) -> str:
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def _short(name: str) -> str:
    name = name.strip('"').replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    cut = name.find("(")
    return name[:cut] if cut > 0 else name[:80]


def trace_table(stats_csv: str) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    out = ["| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| %s | %s | %.1f | %.1f | %.1f | %.2f%% |" % (
            _short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def _counter_rows(path: str, counter: str):
    rows = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def traffic(fetch_csv: str, write_csv: str, copy_mib: int, m: int, n: int, k: int) -> dict:
    copy_bytes = copy_mib * (1 << 20)
    fetch = _counter_rows(fetch_csv, "FETCH_SIZE")
    write = _counter_rows(write_csv, "WRITE_SIZE")
    # the calibration copy: the elementwise kernel with the largest read
    cal_f = max(v for name, v in fetch if "elementwise" in name)
    cal_w = max(v for name, v in write if "elementwise" in name)
    f_factor = copy_bytes / (cal_f * 1024.0)
    w_factor = copy_bytes / (cal_w * 1024.0)
    pf = [v for name, v in fetch if is_product_kernel(name)]
    pw = [v for name, v in write if is_product_kernel(name)]
    fb = sum(pf) / len(pf) * 1024.0 * f_factor
    wb = sum(pw) / len(pw) * 1024.0 * w_factor
    return {"kernel": PRODUCT_KERNEL, "source_sha256_16": source_hash(), "m": m, "n": n, "k": k,
            "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
            "bytes_per_launch": fb + wb, "fetch_scale": f_factor, "write_scale": w_factor,
            "calibration_copy_bytes": copy_bytes, "dispatches": [len(pf), len(pw)]}


def load_traffic(path: str, m: int, n: int, k: int):
    """Bytes per launch from a stored measurement, or None if it does not
    match this shape or the kernel source has changed since."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as fh:
        tr = json.load(fh)
    if (tr.get("m"), tr.get("n"), tr.get("k")) != (m, n, k):
        return None
    if tr.get("source_sha256_16") != source_hash():
        return None
    return tr.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats_csv")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_csv")
    f.add_argument("write_csv")
    f.add_argument("--copy-mib", type=int, required=True)
    f.add_argument("--m", type=int, required=True)
    f.add_argument("--n", type=int, required=True)
    f.add_argument("--k", type=int, required=True)
    f.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "trace":
        print(trace_table(a.stats_csv))
    else:
        res = traffic(a.fetch_csv, a.write_csv, a.copy_mib, a.m, a.n, a.k)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res))


if __name__ == "__main__":
    main()
