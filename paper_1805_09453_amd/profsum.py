"""Summarise rocprofv3 CSV output into a short text report and HBM traffic figures.

    python -m paper_1805_09453_amd.profsum --trace DIR --fetch DIR --write DIR \
        --cmd "<command that produced them>" --out profiles/NAME.md [--traffic profiles/traffic.json] \
        [--logs FETCH_LOG WRITE_LOG]

--trace: a `rocprofv3 --kernel-trace --stats` output directory (kernel_stats.csv);
--fetch / --write: `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` directories
(counter_collection.csv, KiB per dispatch).  The counters are scaled by what they
read for the plain 256 MiB device copy that `bench.py --calib-copy` runs first
(the largest __amd_rocclr_copyBuffer dispatch): scale = 256 MiB / counter value.
Each traffic entry carries the hash of the kernel sources it was measured on
(from the counter runs' own output when --logs is given); bench.py reports the
figure only while the sources still hash the same.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 256 * 1024 * 1024


def _csv(d, suffix):
    f = glob.glob(os.path.join(d, "*" + suffix))
    if not f:
        raise FileNotFoundError(f"no *{suffix} in {d}")
    with open(f[0]) as fh:
        return list(csv.DictReader(fh))


def short(name):
    n = name.replace("(anonymous namespace)::", "")
    m = re.match(r"_ZN12_GLOBAL__N_1\d+(\w+?)E", n)  # a name rocprofv3 left mangled
    if m:
        n = re.sub(r"^\d+", "", m.group(1))
    n = n.split("(")[0]
    n = n.replace("void ", "").replace("gp::", "")
    n = n.replace("HIP_vector_type<float, 2u>", "f32").replace("HIP_vector_type<double, 2u>", "f64")
    return re.sub(r"\s+>", ">", n).strip()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("gprox.hip", "gprox_fft.hpp", "gprox_kernels.hpp", "gprox_fused.hpp", "gprox_generic.hpp",
              "gprox_generic.inc"):
        with open(os.path.join(ROOT, "paper_1805_09453_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_means(rows):
    """(per-kernel steady-state KiB per dispatch, copy-calibration KiB).

    The steady-state figure is the median over the later half of a kernel's
    dispatches (in dispatch order): the timed solve runs last, after the
    launch-shape tuner, whose timing launches run the row kernels in their
    entry mode (fewer stores) and would bias a plain mean."""
    agg, copy = {}, 0.0
    for r in rows:
        v = float(r["Counter_Value"])
        if "copyBuffer" in r["Kernel_Name"]:
            copy = max(copy, v)
        if "gp::" in r["Kernel_Name"]:
            agg.setdefault(short(r["Kernel_Name"]), []).append((int(r.get("Dispatch_Id") or 0), v))
    out = {}
    for k, v in agg.items():
        late = sorted(x for _, x in sorted(v)[len(v) // 2:])
        out[k] = late[len(late) // 2]
    return out, copy


def run_source_hash(logs):
    """The kernel source hash that bench.py printed in both counter runs (they
    must agree): the traffic figures belong to the sources that were measured."""
    hs = set()
    for p in logs:
        with open(p) as fh:
            rows = [json.loads(ln) for ln in fh if ln.startswith("{")]
        if not rows:
            raise ValueError(f"no JSON line in {p}")
        hs.add(rows[-1]["roofline"]["kernel_source_hash"])
    if len(hs) != 1:
        raise ValueError(f"the counter runs measured different sources: {sorted(hs)}")
    return hs.pop()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic")
    ap.add_argument("--title", default="rocprofv3 kernel summary")
    ap.add_argument("--logs", nargs=2, metavar=("FETCH_LOG", "WRITE_LOG"),
                    help="stdout of the two counter runs: the kernel source hash is taken from their JSON lines")
    a = ap.parse_args()

    stats = _csv(a.trace, "kernel_stats.csv")
    lines = [f"# {a.title}", "", "Command:", "", "```", a.cmd, "```", "",
             "| kernel | calls | avg us | total % |", "|---|---:|---:|---:|"]
    for r in stats:
        lines.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    traffic = {}
    if a.fetch and a.write:
        fm, fcopy = counter_means(_csv(a.fetch, "counter_collection.csv"))
        wm, wcopy = counter_means(_csv(a.write, "counter_collection.csv"))
        fs = COPY_BYTES / (fcopy * 1024) if fcopy else 1.0
        ws = COPY_BYTES / (wcopy * 1024) if wcopy else 1.0
        lines += ["", f"HBM bytes per dispatch: FETCH_SIZE x {fs:.3f}, WRITE_SIZE x {ws:.3f} "
                      f"(scales from the 256 MiB copy: it reads {fcopy:.0f} KiB fetch, {wcopy:.0f} KiB write).",
                  "", "| kernel | FETCH KiB | WRITE KiB | HBM MB per dispatch (scaled) |", "|---|---:|---:|---:|"]
        h = run_source_hash(a.logs) if a.logs else kernel_source_hash()
        for k in sorted(set(fm) | set(wm)):
            fb, wb = fm.get(k, 0.0), wm.get(k, 0.0)
            tot = (fb * fs + wb * ws) * 1024
            lines.append(f"| {k} | {fb:.0f} | {wb:.0f} | {tot / 1e6:.1f} |")
            traffic[k] = {"bytes_per_launch": tot, "fetch_kib": fb, "write_kib": wb, "source_hash": h}
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if a.traffic and traffic:
        old = {}
        if os.path.exists(a.traffic):
            with open(a.traffic) as fh:
                old = json.load(fh)
        old.update(traffic)
        with open(a.traffic, "w") as fh:
            json.dump(old, fh, indent=1, sort_keys=True)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
