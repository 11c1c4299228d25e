"""Turn rocprofv3 CSV output into the short summaries kept with the library.

* ``trace``: ``--kernel-trace --stats`` output -> Markdown table of kernels.
* ``traffic``: two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of
  ``bench.py --copy-calibration MIB`` -> HBM bytes per launch of the product
  kernel.  Each counter is scaled by what it reads for the calibration copy
  (an elementwise kernel that reads and writes MIB MiB once), so the figures
  are bytes, whatever unit and coverage the counter has on this GPU.  The
  result records the hash of the kernel source it was taken on; bench.py
  only reports it while that source is unchanged.
* ``counters``: ``--pmc`` runs (SQ, cache, FETCH_SIZE passes) -> per kernel,
  the shader clock it ran at (GRBM_GUI_ACTIVE counts cycles on each of the 8
  XCDs, divided by the dispatch's own duration), the share of SIMD cycles the
  matrix cores were busy (SQ_VALU_MFMA_BUSY_CYCLES over the 1024 SIMDs), the
  same share of 2.4 GHz cycles, the waits per wave cycle, the L2 hit rate and
  the HBM bytes fetched.

Usage::

    python -m paper_2303_04353_amd.profiling trace DIR/run_kernel_stats.csv [--cmd "..."]
    python -m paper_2303_04353_amd.profiling traffic FETCH.csv WRITE.csv --copy-mib 1024 \\
        --m 8192 --n 8192 --k 8192 --out profiles/<name>.json
    python -m paper_2303_04353_amd.profiling counters SQ.csv CACHE.csv FETCH.csv --copy-mib 1024
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# the headline form of the product kernel: no flags, global Sigma and T, 64 x 64
# tiles with seven stored B planes (either staging form: the last template
# argument is left open)
PRODUCT_KERNEL = "cascade_kernel<false, false, Shape<64, 64, 7>"
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
    if not pf or not pw:
        raise ValueError("no dispatch of the product kernel %r in the counter files" % PRODUCT_KERNEL)
    fb = sum(pf) / len(pf) * 1024.0 * f_factor
    wb = sum(pw) / len(pw) * 1024.0 * w_factor
    kname = next(_short(name).replace("ddk::", "") for name, _ in fetch if is_product_kernel(name))
    return {"kernel": kname, "source_sha256_16": source_hash(), "m": m, "n": n, "k": k,
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


# MI355X: 8 XCDs of 32 CUs, 4 SIMDs per CU, 2.4 GHz peak engine clock
XCDS = 8
SIMDS = 256 * 4
PEAK_CLOCK_HZ = 2.4e9


def counter_summary(paths, copy_mib: int = 0) -> dict:
    """Per kernel (short name), counters averaged over its dispatches, plus
    the figures derived from them (see the module docstring).  FETCH_SIZE is
    scaled by the calibration copy when ``copy_mib`` is given."""
    per = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            key = (path, r["Dispatch_Id"])
            d = per.setdefault(key, {"name": _short(r["Kernel_Name"])})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
            d["dur_s"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    fetch_factor = None
    if copy_mib:
        cal = [d["FETCH_SIZE"] for d in per.values()
               if "FETCH_SIZE" in d and "elementwise" in d["name"]]
        if cal:
            fetch_factor = copy_mib * (1 << 20) / (max(cal) * 1024.0)
    groups = {}
    for d in per.values():
        groups.setdefault(d["name"], []).append(d)
    out = {}
    for name, ds in groups.items():
        def total(c, need=()):
            # summed over the dispatches that carry c and every counter in need:
            # ratios of sums weight long dispatches by their length
            return sum(d[c] for d in ds if c in d and all(n in d for n in need))

        m = {}
        for d in ds:
            for c in d:
                if c not in ("name", "dur_s"):
                    m.setdefault(c, []).append(d[c])
        m = {c: sum(v) / len(v) for c, v in m.items()}
        r = {"dispatches": len(ds)}
        both = ("GRBM_GUI_ACTIVE", "SQ_VALU_MFMA_BUSY_CYCLES")
        dur = total("dur_s", both)
        if dur > 0:
            cyc = total("GRBM_GUI_ACTIVE", both) / XCDS
            mfma = total("SQ_VALU_MFMA_BUSY_CYCLES", both)
            r["clock_ghz"] = cyc / dur / 1e9
            r["mfma_busy_of_active"] = mfma / (SIMDS * cyc)
            r["mfma_busy_of_peak_clock"] = mfma / (SIMDS * PEAK_CLOCK_HZ * dur)
        for c in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY"):
            w = total("SQ_WAVE_CYCLES", (c,))
            if w:
                r[c.lower() + "_per_wave_cycle"] = total(c, ("SQ_WAVE_CYCLES",)) / w
        hits, misses = total("TCC_HIT_sum", ("TCC_MISS_sum",)), total("TCC_MISS_sum", ("TCC_HIT_sum",))
        if hits + misses:
            r["l2_hit_rate"] = hits / (hits + misses)
        if "FETCH_SIZE" in m and fetch_factor:
            r["fetch_bytes"] = m["FETCH_SIZE"] * 1024.0 * fetch_factor
        r["counters"] = m
        out[name] = r
    return out


def counter_table(summary: dict, match: str = "") -> str:
    out = ["| kernel | dispatches | clock (GHz) | MFMA busy, of active cycles | "
           "MFMA busy, of 2.4 GHz cycles | SQ_WAIT_ANY / wave cycle | "
           "SQ_WAIT_INST_ANY / wave cycle | L2 hit rate | HBM fetch (GB) |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]

    def f(v, fmt):
        return fmt % v if v is not None else "-"
    for name, r in summary.items():
        if match and match not in name:
            continue
        out.append("| %s | %d | %s | %s | %s | %s | %s | %s | %s |" % (
            name, r["dispatches"], f(r.get("clock_ghz"), "%.2f"),
            f(r.get("mfma_busy_of_active"), "%.3f"), f(r.get("mfma_busy_of_peak_clock"), "%.3f"),
            f(r.get("sq_wait_any_per_wave_cycle"), "%.3f"),
            f(r.get("sq_wait_inst_any_per_wave_cycle"), "%.3f"),
            f(r.get("l2_hit_rate"), "%.3f"),
            f(r["fetch_bytes"] / 1e9 if "fetch_bytes" in r else None, "%.2f")))
    return "\n".join(out)


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
    c = sub.add_parser("counters")
    c.add_argument("csvs", nargs="+")
    c.add_argument("--copy-mib", type=int, default=0)
    c.add_argument("--match", default="")
    a = ap.parse_args()
    if a.cmd == "trace":
        print(trace_table(a.stats_csv))
    elif a.cmd == "counters":
        print(counter_table(counter_summary(a.csvs, a.copy_mib), a.match))
    else:
        res = traffic(a.fetch_csv, a.write_csv, a.copy_mib, a.m, a.n, a.k)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res))


if __name__ == "__main__":
    main()
