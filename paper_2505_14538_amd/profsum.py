"""Summaries of rocprofv3 output for the committed profiles.

Reads the CSV files rocprofv3 writes (``--output-format csv``) and prints or
writes the short summaries kept under ``profiles/``:

* ``kernels``  -- per-kernel time table from ``*_kernel_stats.csv``
                  (``--kernel-trace --stats``), as Markdown;
* ``traffic``  -- HBM bytes per dispatch of the loop and task-build kernels
                  from one ``--pmc FETCH_SIZE`` and one ``--pmc WRITE_SIZE``
                  run, each scaled by what the same counter reads for a
                  plain device copy of known size, as JSON;
* ``valu``     -- FP32 VALU counters per dispatch (FLOPs over 64 lanes per
                  wavefront instruction, instruction mix, lane utilisation)
                  of the same kernels, as JSON.

The JSON files carry a digest of the kernel sources; ``bench.py`` uses a
figure only while the sources still hash to it.

    python -m paper_2505_14538_amd.profsum kernels STATS_CSV
    python -m paper_2505_14538_amd.profsum traffic FETCH_DIR WRITE_DIR \\
        COPY_FETCH_DIR COPY_WRITE_DIR COPY_BYTES OUT_JSON
    python -m paper_2505_14538_amd.profsum valu PMC_DIR OUT_JSON
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))

# kernel-name prefixes the summaries report (all launches of each)
KERNELS = ("k_loop<0", "k_loop<2", "k_tasks<float, 0>", "k_tasks<float, 2>")


def sources_digest() -> str:
    """sha256 over the library's kernel sources (csrc/*.hip, *.h), sorted by name."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _short(name: str) -> str:
    """'void swsph::k_loop<0, float, 512>(...)' -> 'swsph::k_loop<0, float, 512>'."""
    n = name.replace("void ", "", 1)
    return n.split("(")[0]


def _match(name: str, prefix: str) -> bool:
    return _short(name).replace("swsph::", "").startswith(prefix)


def kernel_table(stats_csv: str, top: int = 20) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    out = ["| kernel | calls | total ms | avg ms | min ms | max ms | % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append("| `%s` | %s | %.3f | %.3f | %.3f | %.3f | %.1f |" % (
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6, float(r["MaxNs"]) / 1e6,
            float(r["Percentage"])))
    for prefix in ("k_loop<0", "k_loop<2"):
        sel = [r for r in rows if _match(r["Name"], prefix)]
        if sel:
            calls = sum(int(r["Calls"]) for r in sel)
            tot = sum(float(r["TotalDurationNs"]) for r in sel) / 1e6
            out.append("")
            out.append("`%s, ...>` all launches: %d calls, %.3f ms total, %.3f ms per launch"
                       % (prefix, calls, tot, tot / calls))
    return "\n".join(out)


def _counter_rows(d: str):
    f = glob.glob(os.path.join(d, "*counter_collection.csv"))
    if not f:
        raise SystemExit("no counter_collection.csv in %s" % d)
    return list(csv.DictReader(open(f[0])))


def per_dispatch(d: str, counter: str, prefix: str) -> float:
    """Mean of `counter` over the dispatches of kernels matching prefix."""
    vals = defaultdict(float)
    for r in _counter_rows(d):
        if r["Counter_Name"] == counter and _match(r["Kernel_Name"], prefix):
            vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
    if not vals:
        raise SystemExit("no %s rows for %s in %s" % (counter, prefix, d))
    return sum(vals.values()) / len(vals)


def copy_counter(d: str, counter: str) -> float:
    """Largest per-dispatch value of `counter` among copy kernels (the 1 GiB copies)."""
    best = 0.0
    for r in _counter_rows(d):
        if r["Counter_Name"] == counter and ("copy" in r["Kernel_Name"].lower()
                                              or "elementwise" in r["Kernel_Name"].lower()):
            best = max(best, float(r["Counter_Value"]))
    if best <= 0:
        raise SystemExit("no copy kernel with %s in %s" % (counter, d))
    return best


def traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_bytes, out_json, commands=None):
    kib = copy_bytes / 1024.0
    cf = copy_counter(cfetch_dir, "FETCH_SIZE")
    cw = copy_counter(cwrite_dir, "WRITE_SIZE")
    # a copy reads and writes copy_bytes: scale each counter to that
    f_fac, w_fac = kib / cf, kib / cw
    res = {"workload": "clustered 128^3 (2,097,152 particles), default plan options",
           "method": "FETCH_SIZE and WRITE_SIZE KiB per dispatch (two rocprofv3 --pmc runs), "
                     "scaled by the factors a plain device copy of %d bytes reads for the "
                     "same counters" % copy_bytes,
           "commands": commands or [],
           "copy_factors": {"FETCH_SIZE": f_fac, "WRITE_SIZE": w_fac},
           "sources_sha256": sources_digest(), "kernels": {}}
    for k in KERNELS:
        fk = per_dispatch(fetch_dir, "FETCH_SIZE", k) * f_fac
        wk = per_dispatch(write_dir, "WRITE_SIZE", k) * w_fac
        res["kernels"][k] = {"fetch_bytes": fk * 1024.0, "write_bytes": wk * 1024.0,
                             "bytes_per_dispatch": (fk + wk) * 1024.0}
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    return res


VALU_COUNTERS = ("SQ_INSTS_VALU_FLOPS_FP32", "SQ_INSTS_VALU_FLOPS_FP32_TRANS",
                 "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32",
                 "SQ_INSTS_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_ACTIVE_INST_VALU")


def valu(pmc_dir, out_json, commands=None):
    res = {"workload": "clustered 128^3 (2,097,152 particles), default plan options",
           "method": "one rocprofv3 --pmc run of %s; per-dispatch means over all launches of "
                     "each kernel" % " ".join(VALU_COUNTERS),
           "commands": commands or [], "sources_sha256": sources_digest(), "kernels": {}}
    for k in KERNELS:
        v = {c: per_dispatch(pmc_dir, c, k) for c in VALU_COUNTERS}
        res["kernels"][k] = {
            # the SQ_INSTS counters count wavefront instructions: FLOPs of
            # 64 lanes each (the TOTAL_32_OPS convention), masked lanes included
            "valu_flops_fp32": 64.0 * v["SQ_INSTS_VALU_FLOPS_FP32"],
            "valu_flops_fp32_per_wave_inst": v["SQ_INSTS_VALU_FLOPS_FP32"],
            "valu_flops_fp32_trans": v["SQ_INSTS_VALU_FLOPS_FP32_TRANS"],
            "valu_insts": v["SQ_INSTS_VALU"],
            "fma_f32_insts": v["SQ_INSTS_VALU_FMA_F32"],
            "add_f32_insts": v["SQ_INSTS_VALU_ADD_F32"],
            "mul_f32_insts": v["SQ_INSTS_VALU_MUL_F32"],
            # active lanes per VALU cycle over the 64 of a wavefront
            "lane_utilisation": v["SQ_THREAD_CYCLES_VALU"] / max(1.0, 64.0 * v["SQ_ACTIVE_INST_VALU"]),
            "raw": v}
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    return res


def main(argv):
    if len(argv) < 2:
        raise SystemExit(__doc__)
    cmd = argv[1]
    if cmd == "kernels":
        print(kernel_table(argv[2]))
    elif cmd == "traffic":
        r = traffic(argv[2], argv[3], argv[4], argv[5], int(argv[6]), argv[7])
        print(json.dumps(r["kernels"], indent=1))
    elif cmd == "valu":
        r = valu(argv[2], argv[3])
        print(json.dumps({k: {kk: vv for kk, vv in v.items() if kk != "raw"}
                          for k, v in r["kernels"].items()}, indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv)
