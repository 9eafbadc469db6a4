"""HBM traffic of the smoother kernel from rocprofv3 hardware counters.

Two steps:

1. ``python -m paper_2407_02100_amd.traffic_probe run [--dtype f32|f64]``
   runs on the GPU, under ``rocprofv3 --pmc <COUNTER> --output-format csv``:
   one plain device-to-device copy of a known size (the calibration kernel),
   then one sweep of the smoother on the finest level of the 3D Q4 128^3
   workload (8 color launches).
2. ``python -m paper_2407_02100_amd.traffic_probe summarize FETCH_CSV WRITE_CSV``
   reads the two counter files (FETCH_SIZE and WRITE_SIZE passes, in KiB per
   dispatch), scales each counter by the value it reads for the copy kernel
   (bytes the copy must move / counter), and writes the bytes per smoother
   launch to ``profiles/patch_sweep_traffic.json`` together with a hash of
   the kernel sources (the number is void once the kernel changes).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 512 * 1024 * 1024  # bytes read by the calibration copy (and written)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("patch_wave.h", "patch_impl.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def run(dtype: str, n_cells: int = 128, degree: int = 4):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch
    import vps_inputs as vi
    from paper_2407_02100_amd import vps
    tdt = torch.float32 if dtype == "f32" else torch.float64
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    b = torch.from_numpy(vi.seeded_vector(3, degree, n_cells, 5)).to("cuda", tdt)
    u = torch.from_numpy(vi.seeded_vector(3, degree, n_cells, 105)).to("cuda", tdt)
    with vps.Context(3, degree, n_cells, 1, vcycle_dtype=dtype) as ctx:
        ctx.smooth(0, u, b, sweeps=1)
        ctx.sync()
    print("traffic probe done", flush=True)


def _read(path):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("kernel_name") or ""
        val = float(r.get("Counter_Value") or r.get("counter_value") or 0.0)
        cname = r.get("Counter_Name") or r.get("counter_name") or ""
        did = r.get("Dispatch_Id") or r.get("Correlation_Id") or r.get("dispatch_id") or ""
        out.append((did, name, cname, val))
    return out


def summarize(fetch_csv: str, write_csv: str, dtype: str, workload: str = "poisson3d_q4_n128",
              out_path: str | None = None):
    res = {}
    for label, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _read(path)
        copy = [v for _, n, _, v in rows if "copyBuffer" in n or "copy" in n.lower() and "patch" not in n]
        patch = [v for _, n, _, v in rows if "patch_wave3_kernel" in n or "patch_color_kernel" in n]
        if not copy or not patch:
            raise SystemExit(f"{path}: copy or smoother dispatches missing")
        kib_copy = max(copy)
        scale = COPY_BYTES / (kib_copy * 1024.0)  # bytes per counter KiB-unit
        res[label] = {"copy_kib": kib_copy, "scale": scale,
                      "patch_kib_per_launch": sum(patch) / len(patch),
                      "patch_bytes_per_launch": sum(patch) / len(patch) * 1024.0 * scale,
                      "launches": len(patch)}
    total = res["fetch"]["patch_bytes_per_launch"] + res["write"]["patch_bytes_per_launch"]
    doc = {"workload": workload, "dtype": dtype, "kernel_source_hash": kernel_source_hash(),
           "bytes_per_launch": total, "fetch": res["fetch"], "write": res["write"],
           "note": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE per dispatch, each scaled by the value the "
                   "same counter reads for a plain copy of 512 MiB in the same process"}
    out_path = out_path or os.path.join(ROOT, "profiles", "patch_sweep_traffic.json")
    with open(out_path, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc, indent=1))
    return doc


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--dtype", default="f32")
    s = sub.add_parser("summarize")
    s.add_argument("fetch_csv")
    s.add_argument("write_csv")
    s.add_argument("--dtype", default="f32")
    s.add_argument("--out", default=None)
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.dtype)
    else:
        summarize(a.fetch_csv, a.write_csv, a.dtype, out_path=a.out)
