"""Summaries of rocprofv3 counter runs for the profiles folder.

`python -m paper_1202_6522_amd.counters fp64 <counter_collection.csv> <out.json>`
reads a `rocprofv3 --pmc ... --output-format csv` result of a run of
`bench.py --scalar-only` and writes, per shtn kernel, the median over its
dispatches of each FP64 instruction counter and the FP64 floating-point
operations per launch they imply, tagged with the hash of the kernel's source
file (bench.py uses a summary only while the source is unchanged).

Counting: SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64 count wave instructions; a
wave instruction covers 64 lanes, an FMA is two operations, the others one.
SQ_INSTS_VALU_FLOPS_FP64, where the hardware offers it, is kept as read.

`python -m paper_1202_6522_amd.counters traffic <fetch.csv> <write.csv> <MiB> <out.json>`
reads two such runs (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch) of
`bench.py --scalar-only --calibrate-copy <MiB>` and writes the HBM bytes per
launch of every shtn kernel, each counter scaled by what it reads for the
calibration kernel (torch.neg over <MiB> MiB of float64: reads and writes
<MiB> MiB once).
"""
import collections
import csv
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# kernel name prefix -> (summary key, source file)
KERNELS = {
    "shtn::k_legendre_synth": ("legendre_synth", "legendre.hip"),
    "shtn::k_legendre_analys": ("legendre_analys", "legendre.hip"),
    "shtn::k_c2r": ("c2r", "fft.hip"),
    "shtn::k_r2c": ("r2c", "fft.hip"),
    "shtn::k_prescale": ("prescale", "legendre.hip"),
}


def source_hash(name):
    with open(os.path.join(HERE, "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_key(name):
    base = name.replace("void ", "", 1)
    for prefix, v in KERNELS.items():
        if base.startswith(prefix):
            return v
    return None


def medians(path):
    """{summary key: {counter: median over dispatches of the per-dispatch sum}}"""
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    names = {}
    for r in csv.DictReader(open(path)):
        kv = kernel_key(r["Kernel_Name"])
        if kv is None:
            continue
        per[kv[0]][r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
        names[kv[0]] = kv[1]
    out = {}
    for k, cs in per.items():
        out[k] = {c: statistics.median(d.values()) for c, d in cs.items()}
        out[k]["_source"] = names[k]
    return out


def fp64_summary(path):
    res = {}
    for k, c in medians(path).items():
        fma = c.get("SQ_INSTS_VALU_FMA_F64", 0.0)
        mul = c.get("SQ_INSTS_VALU_MUL_F64", 0.0)
        add = c.get("SQ_INSTS_VALU_ADD_F64", 0.0)
        trans = c.get("SQ_INSTS_VALU_TRANS_F64", 0.0)
        res[k] = {
            "source": c["_source"],
            "source_sha": source_hash(c["_source"]),
            "counters": {n: v for n, v in c.items() if not n.startswith("_")},
            "flops_per_launch": 64.0 * (2.0 * fma + mul + add + trans),
        }
    return res


def calibration_kib(path, counter):
    """Median of `counter` over the dispatches of the calibration kernel."""
    vals = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        if "neg" in r["Kernel_Name"] and r["Counter_Name"] == counter:
            vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
    if not vals:
        raise ValueError("no calibration kernel in %s" % path)
    return statistics.median(vals.values())


def traffic_summary(fetch_csv, write_csv, mib):
    known = mib * 1024.0  # KiB read, and written, by the calibration kernel
    sf = known / calibration_kib(fetch_csv, "FETCH_SIZE")
    sw = known / calibration_kib(write_csv, "WRITE_SIZE")
    fe, wr = medians(fetch_csv), medians(write_csv)
    res = {"_calibration": {"mib": mib, "fetch_scale": sf, "write_scale": sw}}
    for k in sorted(set(fe) & set(wr)):
        fk, wk = fe[k].get("FETCH_SIZE", 0.0), wr[k].get("WRITE_SIZE", 0.0)
        res[k] = {"source": fe[k]["_source"], "source_sha": source_hash(fe[k]["_source"]),
                  "fetch_kib": fk, "write_kib": wk,
                  "bytes_per_launch": int(round(1024.0 * (fk * sf + wk * sw)))}
    return res


def main(argv):
    if len(argv) == 4 and argv[1] == "fp64":
        res = fp64_summary(argv[2])
        with open(argv[3], "w") as f:
            json.dump(res, f, indent=1, sort_keys=True)
        for k, v in sorted(res.items()):
            print("%-16s %.4g FP64 ops per launch" % (k, v["flops_per_launch"]))
        return 0
    if len(argv) == 6 and argv[1] == "traffic":
        res = traffic_summary(argv[2], argv[3], float(argv[4]))
        with open(argv[5], "w") as f:
            json.dump(res, f, indent=1, sort_keys=True)
        for k, v in sorted(res.items()):
            if not k.startswith("_"):
                print("%-16s %.2f MB per launch" % (k, v["bytes_per_launch"] / 1e6))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv))
