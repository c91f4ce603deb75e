"""HBM traffic of the apply kernels from hardware byte counters.

rocprofv3 --pmc writes one CSV row per (dispatch, counter).  FETCH_SIZE and
WRITE_SIZE read the bytes the L2 fetched from and wrote to memory; their unit
and coverage are calibrated here against the plain copy kernel k_copy16 of a
known size that runs in the same process: factor = bytes it moved / counter
reading.  A traffic record stores the digest of the kernel sources it was
measured on (and of the plan layout, which sets the bytes), so a changed kernel
invalidates it; a record file holds one
record per kernel and plan configuration.

    python -m paper_math_0610051_amd.pmc FETCH.csv WRITE.csv --copy-bytes B \
        --kernel k_interp --out record.json [--meta key=value ...]
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
KERNEL_SOURCES = ("apply.hip", "apply.hpp", "common.hpp", "fft.hpp", "interp_util.hpp", "plan.hpp", "plan.hip")


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace collapsed, so that an
    edit of comments alone leaves the digest unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":  # string or character literal, copied whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_digest() -> str:
    """sha256 over the code (comments stripped) of the apply kernels' sources."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), encoding="utf-8") as f:
            h.update(name.encode() + b"\0" + _code_only(f.read()).encode())
    return h.hexdigest()


def read_counter(path, counter):
    """{kernel short name: [value per dispatch in dispatch order]} for one counter."""
    rows = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            short = name.split("(")[0].split("<")[0].split("::")[-1].replace("void ", "").strip()
            rows.setdefault(short, []).append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    return {k: [v for _, v in sorted(vs)] for k, vs in rows.items()}


def traffic_record(fetch_csv, write_csv, copy_bytes, kernel, meta=None):
    fetch = read_counter(fetch_csv, "FETCH_SIZE")
    write = read_counter(write_csv, "WRITE_SIZE")
    for tab, cname in ((fetch, "FETCH_SIZE"), (write, "WRITE_SIZE")):
        if "k_copy16" not in tab or kernel not in tab:
            raise SystemExit("%s: no k_copy16 or %s dispatches" % (cname, kernel))
    f_copy = sum(fetch["k_copy16"]) / len(fetch["k_copy16"])
    w_copy = sum(write["k_copy16"]) / len(write["k_copy16"])
    f_scale, w_scale = copy_bytes / f_copy, copy_bytes / w_copy
    fk = sum(fetch[kernel]) / len(fetch[kernel])
    wk = sum(write[kernel]) / len(write[kernel])
    rec = dict(kernel=kernel, source_digest=source_digest(), copy_bytes=copy_bytes,
               fetch_counter_per_copy=f_copy, write_counter_per_copy=w_copy,
               fetch_scale=f_scale, write_scale=w_scale,
               dispatches=[len(fetch[kernel]), len(write[kernel])],
               fetch_bytes=fk * f_scale, write_bytes=wk * w_scale,
               traffic_bytes=fk * f_scale + wk * w_scale,
               others={k: dict(fetch_bytes=sum(v) / len(v) * f_scale,
                               write_bytes=(sum(write[k]) / len(write[k]) * w_scale) if k in write else None)
                       for k, v in fetch.items() if k not in (kernel, "k_copy16")})
    rec.update(meta or {})
    return rec


def _records(path):
    """The records of a traffic file: {"records": [...]}, or one bare record."""
    if not path or not os.path.exists(path):
        return []
    with open(path) as f:
        data = json.load(f)
    return data.get("records", []) if "records" in data else [data]


def load_traffic(path, kernel, **expect):
    """Traffic bytes per launch from the stored record of this kernel and plan
    configuration (expect: N, B, L, sigma, ...), or None if absent or stale."""
    digest = source_digest()
    for rec in _records(path):
        if rec.get("kernel") != kernel or rec.get("source_digest") != digest:
            continue
        if all(rec.get(k) == v for k, v in expect.items()):
            return rec
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--copy-bytes", type=float, required=True)
    ap.add_argument("--kernel", default="k_interp")
    ap.add_argument("--out", required=True)
    ap.add_argument("--meta", nargs="*", default=[])
    a = ap.parse_args()
    meta = {}
    for kv in a.meta:
        k, v = kv.split("=", 1)
        try:
            v = json.loads(v)
        except ValueError:
            pass
        meta[k] = v
    rec = traffic_record(a.fetch_csv, a.write_csv, a.copy_bytes, a.kernel, meta)
    # one record per kernel and plan configuration: a new one replaces the
    # record of the same configuration, stale or not
    key = lambda r: json.dumps({k: r.get(k) for k in ["kernel"] + sorted(meta)}, sort_keys=True)
    recs = [r for r in _records(a.out) if key(r) != key(rec)] + [rec]
    with open(a.out, "w") as f:
        json.dump({"records": recs}, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
