#!/usr/bin/env python3
"""HBM traffic of the bench's kernels from rocprofv3 counters.

Takes four rocprofv3 `--pmc` runs (each a directory with
`run_counter_collection.csv`):
  --copy-fetch / --copy-write : FETCH_SIZE / WRITE_SIZE of `bench.py --calibrate-copy`
                                (a plain device copy of a known 512 MiB)
  --fetch / --write           : FETCH_SIZE / WRITE_SIZE of the bench command
and writes profiles/traffic_<name>.json: bytes per frame read and written by
each kernel, each counter scaled by (true bytes / counter bytes) of the copy.
The file records a fingerprint of the kernel sources; bench.py reports the
traffic only while the sources are unchanged.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["paper_2204_02348_amd/csrc/dh_kernels.hip", "paper_2204_02348_amd/csrc/dh_fft.hpp"]
COPY_BYTES = 512 * 1024 * 1024


def source_fingerprint() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(d):
    path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    return list(csv.DictReader(open(path)))


def per_kernel(d, counter):
    """{kernel name: (sum of the counter in KB, dispatch count, grid sizes)}"""
    acc = collections.defaultdict(lambda: [0.0, 0])
    for r in _rows(d):
        if r["Counter_Name"] != counter:
            continue
        k = r["Kernel_Name"].split("(")[0].replace("void ", "")
        acc[k][0] += float(r["Counter_Value"])
        acc[k][1] += 1
    return acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--frames-per-launch", type=int, required=True,
                    help="frames each launch of the bench's kernels processes")
    ap.add_argument("--name", required=True)
    ap.add_argument("--command", required=True, help="the profiled command, recorded in the output")
    a = ap.parse_args()
    cf = sum(v[0] for k, v in per_kernel(a.copy_fetch, "FETCH_SIZE").items() if "copy" in k.lower())
    cw = sum(v[0] for k, v in per_kernel(a.copy_write, "WRITE_SIZE").items() if "copy" in k.lower())
    f_scale = COPY_BYTES / (cf * 1024)
    w_scale = COPY_BYTES / (cw * 1024)
    fetch = per_kernel(a.fetch, "FETCH_SIZE")
    write = per_kernel(a.write, "WRITE_SIZE")
    # each counter run is averaged over its own dispatches (the two runs can
    # process different batch counts: the bench's clock settling is timed)
    fpl = a.frames_per_launch
    kernels = {}
    for k in fetch:
        w = write.get(k, [0.0, 1])
        kernels[k] = {
            "read_bytes_per_frame": fetch[k][0] / fetch[k][1] * 1024 * f_scale / fpl,
            "write_bytes_per_frame": w[0] / max(w[1], 1) * 1024 * w_scale / fpl,
            "dispatches": [fetch[k][1], w[1]],
        }
    out = {"name": a.name, "fingerprint": source_fingerprint(), "fetch_scale": f_scale, "write_scale": w_scale,
           "copy_counter_kb": {"FETCH_SIZE": cf, "WRITE_SIZE": cw, "copy_bytes": COPY_BYTES},
           "frames_per_launch": fpl, "command": a.command, "kernels": kernels}
    path = os.path.join(HERE, "profiles", f"traffic_{a.name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
