"""Workload for the HBM traffic counters of the solver kernels.

Run under rocprofv3 with one counter per pass, for example

    rocprofv3 --pmc FETCH_SIZE -d OUT --output-format csv -- python3 paper_1501_04840_amd/profile_traffic.py
    rocprofv3 --pmc WRITE_SIZE -d OUT --output-format csv -- python3 paper_1501_04840_amd/profile_traffic.py

With the argument ``hue`` it runs the hue rendering workload of bench.py
instead (three calls of 33 frames of a 3840 x 2160 image).  By default it
runs 70 iterations of the 256 x 256 x 3 x 32 workload (past the refined
start of the default projection mode, so the steady-state kernels are
counted) and then a plain
elementwise copy of known size (256 MiB read, 256 MiB written), whose
counter values calibrate the solver kernels' readings, and an add of two
such arrays, whose calibrated reading checks the scales on a kernel with
two read streams.  ``summarise`` turns
the two counter CSVs into bytes per launch per kernel.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COPY_ELEMS = 64 * 1024 * 1024          # float32 elements of the calibration copy


def run(iters: int = 70, size=(256, 256, 3, 32)):
    import torch
    from paper_1501_04840_amd import otdyn
    from synth import inputs
    X, Y, C, P = size
    f0, f1 = inputs.cfg3_pair(X, Y)
    d = otdyn.ot_dyn_default_desc(X, Y, C, P)
    prob = otdyn.Problem(d, "cuda:0")
    prob.set_boundary(torch.from_numpy(f0), torch.from_numpy(f1))
    prob.init(otdyn.OT_INIT_COLD)
    prob.step(iters)
    torch.cuda.synchronize()
    _calibration_kernels(torch)
    prob.close()
    print("profile_traffic: done", flush=True)


def _calibration_kernels(torch):
    """The copy that calibrates the counters (COPY_ELEMS floats read and
    written), then an add of two such arrays into a third, whose calibrated
    reading is checked against its own known bytes (two read streams, one
    write stream)."""
    src = torch.rand(COPY_ELEMS, device="cuda:0")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    src2 = torch.rand(COPY_ELEMS, device="cuda:0")
    torch.add(src, src2, out=dst)
    torch.cuda.synchronize()


def _sources_hash() -> str:
    """Hash of the solver's kernel sources (the hue image pipeline's kernels
    are not part of this workload)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1501_04840_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f == "hue.hip":
            continue
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def run_hue(H: int = 2160, W: int = 3840, n: int = 360, frames: int = 33, calls: int = 3):
    """The hue rendering workload as bench.py times it (calls of `frames`
    frames on one 3840 x 2160 image), then the calibration copy."""
    import numpy as np
    import torch
    from paper_1501_04840_amd import othue
    from synth import inputs
    img = inputs.hue_image(501, H, W, sigma=24.0)
    dens = np.stack([inputs.von_mises_hist(600 + i, n) for i in range(frames)]).astype(np.float32)
    r = othue.HueRenderer(H * W, n)
    r.set_source(torch.from_numpy(img.reshape(-1).copy()).cuda())
    tg = torch.from_numpy(dens).cuda()
    out = torch.empty(frames, H * W, 3, dtype=torch.uint8, device="cuda")
    for _ in range(calls):
        othue.ot_hue_render(r.h, tg, frames, out)
    torch.cuda.synchronize()
    _calibration_kernels(torch)
    r.close()
    print("profile_traffic hue: done", flush=True)


def hue_sources_hash() -> str:
    """Hash of the hue image pipeline's kernel source."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1501_04840_amd", "csrc", "hue.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def _kernel_name(raw: str) -> str:
    return raw.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")


def _read(dirname: str, counter: str):
    """{kernel name: [value per dispatch]} from a rocprofv3 counter CSV."""
    files = glob.glob(os.path.join(dirname, "**", "*counter_collection.csv"), recursive=True)
    out = {}
    for fn in files:
        with open(fn) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                name = _kernel_name(row["Kernel_Name"])
                out.setdefault(name, []).append(float(row["Counter_Value"]))
    return out


def summarise(fetch_dir: str, write_dir: str, out_json: str, out_md: str, cmd: str,
              workload: str = "rgb"):
    """workload "rgb": the solver kernels of the 256 x 256 x 3 x 32 run;
    "hue": the hue pipeline kernels of the 3840 x 2160 rendering run."""
    fetch = _read(fetch_dir, "FETCH_SIZE")
    write = _read(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "AUnaryFunctor" in k or "MulFunctor" in k]
    if not copy:
        raise SystemExit("calibration copy kernel not found")
    ck = copy[0]
    nbytes = COPY_ELEMS * 4
    # counters are in KiB per dispatch; scale so the copy reads and writes nbytes
    f_scale = nbytes / (max(fetch[ck]) * 1024.0)
    w_scale = nbytes / (max(write[ck]) * 1024.0)
    check = None
    add = [k for k in fetch if "add" in k.lower() and ("Functor" in k or "functor" in k)
           and k != ck]
    if add and add[0] in write:
        ak = add[0]
        check = {"kernel": ak, "fetch_expected": 2 * nbytes, "write_expected": nbytes,
                 "fetch_calibrated": max(fetch[ak]) * 1024.0 * f_scale,
                 "write_calibrated": max(write[ak]) * 1024.0 * w_scale}
    kernels = {}
    hue = workload == "hue"
    for k in fetch:
        if not (k.startswith(("k_hue_", "k_sort_")) if hue else k.startswith("otd::")):
            continue
        fv = sum(fetch[k]) / len(fetch[k]) * 1024.0 * f_scale
        wv = sum(write.get(k, [0.0])) / max(1, len(write.get(k, []))) * 1024.0 * w_scale
        kernels[k.replace("otd::", "")] = {"fetch_bytes": fv, "write_bytes": wv,
                                           "bytes_per_launch": fv + wv,
                                           "dispatches": len(fetch[k])}
    title = ("hue rendering 3840x2160, 360 bins, 33 frames per launch" if hue
             else "RGB transport 256x256x3x32")
    res = {"sources": hue_sources_hash() if hue else _sources_hash(),
           "workload": "hue_render_3840x2160_360" if hue else "rgb_256x256x3x32",
           "calibration": {"kernel": ck, "bytes_each_way": nbytes,
                           "fetch_scale": f_scale, "write_scale": w_scale,
                           "check": check},
           "kernels": kernels}
    with open(out_json, "w") as fh:
        json.dump(res, fh, indent=1)
    lines = [f"# HBM traffic per launch: {title}", "",
             "Commands (repository root, one MI355X):", "", f"    {cmd}", "",
             f"Calibration: `{ck}` copies {nbytes} B each way; FETCH_SIZE scale "
             f"{f_scale:.4f}, WRITE_SIZE scale {w_scale:.4f}."]
    if check:
        lines[-1] += (f" Check: `{check['kernel']}` (reads {2 * nbytes} B, writes {nbytes} B) "
                      f"reads {check['fetch_calibrated'] / check['fetch_expected']:.4f} and "
                      f"writes {check['write_calibrated'] / check['write_expected']:.4f} of its "
                      "bytes under the same scales.")
    lines += ["",
             "| kernel | fetch MB | write MB | total MB / launch |", "|---|---|---|---|"]
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch"]):
        lines.append(f"| `{k}` | {v['fetch_bytes'] / 1e6:.1f} | {v['write_bytes'] / 1e6:.1f} | "
                     f"{v['bytes_per_launch'] / 1e6:.1f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarise_stats(stats_csv: str, out_md: str, title: str, cmd: str, note: str = "",
                    top: int = 16):
    """Markdown table of a rocprofv3 --stats kernel summary (kernel_stats.csv)."""
    with open(stats_csv) as fh:
        rows = list(csv.DictReader(fh))
    lines = [f"# {title}", "", "Command (repository root, one MI355X):", "", f"    {cmd}", ""]
    if note:
        lines += [note, ""]
    lines += ["| kernel | calls | avg us | min us | max us | total % |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarise_counters(dirname: str, counters, out_md: str, title: str, cmd: str,
                       prefix: str = "otd::", note: str = ""):
    """Markdown table of instruction / wait counters (rocprofv3 --pmc, one run)
    per kernel: the average per dispatch of each counter, and per wave where
    SQ_WAVES was collected."""
    vals = {c: _read(dirname, c) for c in counters}
    names = sorted({k for c in counters for k in vals[c] if k.startswith(prefix)})
    lines = [f"# {title}", "", "Command (repository root, one MI355X):", "", f"    {cmd}", ""]
    if note:
        lines += [note, ""]
    per_wave = "SQ_WAVES" in counters
    head = ["kernel", "dispatches"] + [c + (" / wave" if per_wave and c != "SQ_WAVES" else "")
                                       for c in counters]
    lines += ["| " + " | ".join(head) + " |", "|" + "---|" * len(head)]
    for k in names:
        row = [f"`{k.replace(prefix, '')}`", str(len(vals[counters[0]].get(k, [])))]
        waves = (sum(vals["SQ_WAVES"][k]) / len(vals["SQ_WAVES"][k])) if per_wave and k in vals["SQ_WAVES"] else None
        for c in counters:
            v = vals[c].get(k)
            if not v:
                row.append("-")
                continue
            m = sum(v) / len(v)
            if per_wave and c != "SQ_WAVES" and waves:
                m /= waves
            row.append(f"{m:.1f}")
        lines.append("| " + " | ".join(row) + " |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1:] == ["hue"]:
        run_hue()
    else:
        run()
