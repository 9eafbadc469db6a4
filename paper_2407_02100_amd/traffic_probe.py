"""HBM traffic of the smoother kernel from rocprofv3 hardware counters.

Two steps:

1. ``python -m paper_2407_02100_amd.traffic_probe run [--dtype f32|f64] [--algorithm combined|separated]``
   runs on the GPU, under ``rocprofv3 --pmc <COUNTER> --output-format csv``:
   one plain device-to-device copy of a known size (the calibration kernel),
   then one sweep of the smoother on one 3D level (default: the finest level
   of the 3D Q4 128^3 workload; ``--degree``, ``--cells`` pick another):
   8 color steps, one kernel each for the combined form, a residual and a
   solve kernel each for the separated form.
2. ``python -m paper_2407_02100_amd.traffic_probe summarize FETCH_CSV WRITE_CSV [--out FILE]``
   reads the two counter files (FETCH_SIZE and WRITE_SIZE passes, in KiB per
   dispatch), scales each counter by the value it reads for the copy kernel
   (bytes the copy must move / counter), and writes the bytes per launch of
   every smoother kernel and per sweep (by default to
   ``profiles/patch_sweep_traffic.json``) together with a hash of the kernel
   sources (the number is void once the kernel changes).
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


def strip_comments(src: str) -> str:
    """C/C++ source without its comments (string and character literals kept), each comment
    replaced by one space: what the compiler sees."""
    out = []
    i, n = 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return "".join(out)


def kernel_source_hash() -> str:
    """Hash of every library source (kernels, launchers, host driver) and the C header, comments
    left out: a traffic profile taken with other code is void, whichever file changed the kernel or
    its launch; a change to the comments alone keeps it."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    files = sorted(f for f in os.listdir(csrc) if f.endswith((".h", ".hip", ".cpp")))
    for f in files + [os.path.join("..", "..", "include", "vps.h")]:
        h.update(f.encode())
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def run(dtype: str, n_cells: int = 128, degree: int = 4, algorithm: str = "combined", order: int = 0,
        batch_layers: int = 0, patches_per_wave: int = 0):
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
    with vps.Context(3, degree, n_cells, 1, vcycle_dtype=dtype, algorithm=algorithm, patch_order=order,
                     batch_layers=batch_layers, patches_per_wave=patches_per_wave) as ctx:
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


SMOOTHER_KERNELS = ("patch_wave3_kernel", "patch_pair3_kernel", "patch_row3_kernel", "patch_row5_kernel",
                    "patch_big3_kernel", "patch_color_kernel", "patch_solve3_kernel", "stream3_kernel")


def summarize(fetch_csv: str, write_csv: str, dtype: str, workload: str = "poisson3d_q4_n128",
              out_path: str | None = None, batch_layers: int = 0):
    per = {}
    scales = {}
    for label, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _read(path)
        copy = [v for _, n, _, v in rows if "copyBuffer" in n or "copy" in n.lower() and "patch" not in n]
        if not copy:
            raise SystemExit(f"{path}: copy dispatch missing")
        kib_copy = max(copy)
        scale = COPY_BYTES / (kib_copy * 1024.0)  # bytes per counter KiB-unit
        scales[label] = {"copy_kib": kib_copy, "scale": scale}
        for _, n, _, v in rows:
            key = next((k for k in SMOOTHER_KERNELS if k in n), None)
            if key:
                per.setdefault(key, {}).setdefault(label, []).append(v * 1024.0 * scale)
    if not per:
        raise SystemExit("no smoother dispatches in the counter files")
    kernels = {}
    for key, d in per.items():
        f, w = d.get("fetch", [0.0]), d.get("write", [0.0])
        kernels[key] = {"launches": len(f), "fetch_bytes_per_launch": sum(f) / len(f),
                        "write_bytes_per_launch": sum(w) / len(w)}
    sweep = sum((v["fetch_bytes_per_launch"] + v["write_bytes_per_launch"]) * v["launches"] for v in kernels.values())
    doc = {"workload": workload, "dtype": dtype, "batch_layers": batch_layers, "kernel_source_hash": kernel_source_hash(),
           "kernels": kernels, "bytes_per_sweep": sweep, "calibration": scales,
           "note": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE per dispatch, each scaled by the value the "
                   "same counter reads for a plain copy of 512 MiB in the same process"}
    main = next((kernels[k] for k in ("patch_row3_kernel", "patch_row5_kernel", "patch_big3_kernel",
                                      "patch_wave3_kernel", "patch_pair3_kernel", "patch_color_kernel")
                 if k in kernels), None)
    if main:
        doc["bytes_per_launch"] = main["fetch_bytes_per_launch"] + main["write_bytes_per_launch"]
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
    r.add_argument("--algorithm", default="combined")
    r.add_argument("--order", type=int, default=0, help="vps_config.patch_order")
    r.add_argument("--batch-layers", type=int, default=0, help="vps_config.batch_layers")
    r.add_argument("--degree", type=int, default=4, help="Q_k degree of the 3D level swept")
    r.add_argument("--cells", type=int, default=128, help="cells per direction of the 3D level swept")
    r.add_argument("--ppw", type=int, default=0, help="vps_config.patches_per_wave")
    s = sub.add_parser("summarize")
    s.add_argument("fetch_csv")
    s.add_argument("write_csv")
    s.add_argument("--dtype", default="f32")
    s.add_argument("--out", default=None)
    s.add_argument("--batch-layers", type=int, default=0, help="the batch_layers the counters were taken with")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.dtype, n_cells=a.cells, degree=a.degree, algorithm=a.algorithm, order=a.order,
            batch_layers=a.batch_layers, patches_per_wave=a.ppw)
    else:
        summarize(a.fetch_csv, a.write_csv, a.dtype, out_path=a.out, batch_layers=a.batch_layers)
