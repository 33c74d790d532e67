"""HBM traffic of one kernel from rocprofv3 hardware counters.

Two counter runs of the same command give FETCH_SIZE and WRITE_SIZE (KiB per
dispatch, summed over the L2 channels).  The counters are scaled to bytes by a
plain device-to-device copy of known size profiled the same way
(`bench.py --copy-probe`, which reads and writes 1 GiB per launch): factor =
known bytes / counted bytes, separately for reads and writes.  The result is
written as a small JSON record next to the profile summaries; it carries the
SHA-256 of the kernel's source file, so a reader can tell whether the kernel
has changed since the counters were taken.

    python -m paper_2108_08845_amd.pmc_traffic \\
        --fetch RUN_DIR --write RUN_DIR --copy-fetch RUN_DIR --copy-write RUN_DIR \\
        --kernel 'k_sketch_bf16<32, 10>' --kclass fused_bf16 --workload NAME --out FILE.json

RUN_DIR is a rocprofv3 output directory written with --output-format csv
(its *counter_collection.csv files are read).
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {
    "fused_bf16": os.path.join(HERE, "csrc", "panel.hip"),
    "fused_f32": os.path.join(HERE, "csrc", "panel.hip"),
    "lift": os.path.join(HERE, "csrc", "panel.hip"),
    "split": os.path.join(HERE, "csrc", "panel.hip"),
    "split3": os.path.join(HERE, "csrc", "panel.hip"),
    "tn": os.path.join(HERE, "csrc", "panel.hip"),
}
COPY_BYTES = 1 << 30


def source_sha256(kclass):
    path = KERNEL_SOURCES.get(kclass)
    if path is None or not os.path.exists(path):
        return None
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def read_counters(run_dir, counter):
    """{kernel name: [value per dispatch]} for one counter of a csv run."""
    out = {}
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *counter_collection.csv under {run_dir}")
    per_dispatch = {}
    for fn in files:
        with open(fn, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                key = (fn, row.get("Dispatch_Id") or row.get("Correlation_Id"))
                name = row.get("Kernel_Name", "")
                v = float(row["Counter_Value"])
                # a counter may be reported per dimension (e.g. per channel): sum them
                if key in per_dispatch:
                    per_dispatch[key][1] += v
                else:
                    per_dispatch[key] = [name, v]
    for name, v in per_dispatch.values():
        out.setdefault(name, []).append(v)
    return out


def pick(counters, substr):
    hits = {k: v for k, v in counters.items() if substr in k}
    if not hits:
        raise KeyError(f"no kernel matching {substr!r}; kernels: {sorted(counters)[:20]}")
    if len(hits) > 1:
        # the most frequent match (e.g. several template instances of one kernel)
        name = max(hits, key=lambda k: len(hits[k]))
    else:
        name = next(iter(hits))
    vals = hits[name]
    return name, sum(vals) / len(vals), len(vals)


def copy_kernel(counters):
    """The copy launches: the kernel with the largest counter value per dispatch."""
    name = max(counters, key=lambda k: max(counters[k]))
    vals = counters[name]
    return name, sum(vals) / len(vals), len(vals)


def compute(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, kernel, kclass, workload):
    fk_name, fk, nf = pick(read_counters(fetch_dir, "FETCH_SIZE"), kernel)
    wk_name, wk, nw = pick(read_counters(write_dir, "WRITE_SIZE"), kernel)
    cf_name, cf, _ = copy_kernel(read_counters(copy_fetch_dir, "FETCH_SIZE"))
    cw_name, cw, _ = copy_kernel(read_counters(copy_write_dir, "WRITE_SIZE"))
    f_fetch = COPY_BYTES / (cf * 1024.0)
    f_write = COPY_BYTES / (cw * 1024.0)
    fetch_b = fk * 1024.0 * f_fetch
    write_b = wk * 1024.0 * f_write
    return {
        "kernel": fk_name, "class": kclass, "workload": workload,
        "source_sha256": source_sha256(kclass),
        "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "dispatches": [nf, nw],
        "copy_kernel": cf_name, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "factor_fetch": f_fetch, "factor_write": f_write,
        "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
        "traffic_bytes_per_launch": fetch_b + write_b,
    }


def load_current(profiles_dir, kclass, workload):
    """Traffic record for (kclass, workload) whose source hash matches the current source, else None."""
    sha = source_sha256(kclass)
    for fn in sorted(glob.glob(os.path.join(profiles_dir, "*.json"))):
        try:
            with open(fn) as f:
                rec = json.load(f)
        except (OSError, ValueError):
            continue
        if rec.get("class") == kclass and rec.get("workload") == workload and rec.get("source_sha256") == sha:
            return rec
    return None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--kclass", required=True, choices=sorted(KERNEL_SOURCES))
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", action="append", default=[],
                    help="a command that produced the counter runs (repeatable; stored in the record)")
    a = ap.parse_args(argv)
    rec = compute(a.fetch, a.write, a.copy_fetch, a.copy_write, a.kernel, a.kclass, a.workload)
    if a.command:
        rec["commands"] = list(a.command)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    json.dump(rec, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main()
