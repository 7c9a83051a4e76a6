"""Short text summaries of rocprofv3 CSV output for the sweep kernel.

  python -m paper_1910_08448_amd.rocprof_summary stats DIR
      kernel table (calls, average / min / max duration, share) from DIR/run_kernel_stats.csv
  python -m paper_1910_08448_amd.rocprof_summary pmc DIR [DIR ...]
      mean counter value per dispatch of the sweep kernels and of the copy probe
  python -m paper_1910_08448_amd.rocprof_summary valu DIR UPDATES
      VALU issue of the sweep kernels from a run with SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU,
      SQ_ACTIVE_INST_VALU2, SQ_INSTS_VALU_TRANS_F32 and GRBM_GUI_ACTIVE: issue units (quad-cycles
      of VALU work; a transcendental takes two) per quad-cycle per SIMD over the kernel's active
      time -- against one (single issue) and two (the dual-issue limit) --, the share of
      quad-cycles that issued two instructions, and lane-units and transcendentals per site
      update (UPDATES = site updates per launch of the inference sweep)
  python -m paper_1910_08448_amd.rocprof_summary traffic KEY COPY_MIB FETCH_DIR WRITE_DIR [OUT]
      HBM bytes per launch of the inference sweep kernel: FETCH_SIZE and WRITE_SIZE (KiB per
      dispatch) each scaled by what the same counter read for the copy probe of COPY_MIB MiB
      read + COPY_MIB MiB written; merged into OUT (JSON) under KEY (workload/precision)
      together with a digest of the kernel sources, so a later kernel change voids the entry.

The directories are rocprofv3 `--output-format csv -o run` output directories.
"""
import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("mpr_device.hpp", "mpr_sparse.hpp", "mpr_tiled.hpp", "mpr.hip"):
        with open(os.path.join(ROOT, "paper_1910_08448_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _infer_sweep_kind(name):
    """Which inference-sweep kernel a dispatch is: 'fused' (k_sweep with energy sums in double
    precision), 'tiled' (k_tiled), 'sparse0' / 'sparse1' (the compacted path's colour kernels),
    or None."""
    if "k_sweep" in name and ("1, false" in name or "Li1ELb0" in name):
        return "fused"
    if "k_tiled" in name and (re.search(r"k_tiled<[^,<>]+, [^,<>]+, 1, (false|true)[,>]", name) or
                              "Li1ELb0E" in name or "Li1ELb1E" in name):
        return "tiled"
    if "k_sparse" in name:
        for c in (0, 1):
            if ", 1, false, %d>" % c in name or ", 1, true, %d>" % c in name or \
               "Li1ELb0ELi%dE" % c in name or "Li1ELb1ELi%dE" % c in name:
                return "sparse%d" % c
    return None


def _is_copy(row):
    return "copyBuffer" in row["Kernel_Name"] and int(row["Grid_Size"]) > 100000


def _probe_dispatch(rows):
    """The copy probe is the first large device copy of the run (bench.py --copy-probe-mib
    issues it before anything else)."""
    ids = [int(r["Dispatch_Id"]) for r in rows if _is_copy(r)]
    return min(ids) if ids else None


def stats(d, top=10):
    rows = list(csv.DictReader(open(os.path.join(d, "run_kernel_stats.csv"))))
    out = ["| kernel | calls | avg µs | min µs | max µs | % |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append("| `%s` | %s | %.2f | %.2f | %.2f | %.1f |" % (
            r["Name"][:90], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def _pmc_means(dirs):
    agg = collections.defaultdict(list)
    for d in dirs:
        rows = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
        probe = _probe_dispatch(rows)
        for r in rows:
            if _is_copy(r):
                if int(r["Dispatch_Id"]) != probe:
                    continue
                name = "copy probe"
            elif any(k in r["Kernel_Name"] for k in ("k_sweep", "k_sparse", "k_tiled")):
                name = r["Kernel_Name"][:70]
            else:
                continue
            agg[(name, r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}, {k: len(v) for k, v in agg.items()}


def pmc(dirs):
    means, counts = _pmc_means(dirs)
    out = ["| kernel | counter | dispatches | mean per dispatch |", "|---|---|---|---|"]
    for (k, c) in sorted(means):
        out.append("| `%s` | %s | %d | %.6g |" % (k, c, counts[(k, c)], means[(k, c)]))
    return "\n".join(out)


N_SIMD = 256 * 4          # MI355X: 256 CUs x 4 SIMDs
N_XCD = 8                 # GRBM_GUI_ACTIVE is reported summed over the 8 XCDs


def valu(d, updates):
    rows = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        k = _infer_sweep_kind(r["Kernel_Name"])
        if k is None:
            if "k_sweep" in r["Kernel_Name"] or "k_tiled" in r["Kernel_Name"] or "k_sparse" in r["Kernel_Name"]:
                k = "other sweep variant: " + r["Kernel_Name"][:60]
            else:
                continue
        agg[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = ["| kernel | dispatches | VALU instr / dispatch | issue units / quad-cycle / SIMD | of single issue | of dual issue | dual-issued quad-cycles | lane-units / update | transcendentals / update |",
           "|---|---|---|---|---|---|---|---|---|"]
    for k in sorted(agg):
        m = {c: sum(v) / len(v) for c, v in agg[k].items()}
        n = len(agg[k].get("SQ_INSTS_VALU", []))
        act, act2 = m.get("SQ_ACTIVE_INST_VALU", 0.0), m.get("SQ_ACTIVE_INST_VALU2", 0.0)
        quads = m.get("GRBM_GUI_ACTIVE", 0.0) / N_XCD / 4.0
        rate = act / (N_SIMD * quads) if quads else float("nan")
        per_upd = act * 64.0 / updates if k in ("fused", "tiled") else float("nan")
        tr = m.get("SQ_INSTS_VALU_TRANS_F32", 0.0) * 64.0 / updates if k in ("fused", "tiled") else float("nan")
        out.append("| %s | %d | %.4g | %.3f | %.3f | %.3f | %.3f | %.1f | %.2f |" % (
            k, n, m.get("SQ_INSTS_VALU", 0.0), rate, rate, rate / 2.0, act2 / act if act else 0.0, per_upd, tr))
    # the compacted path's sweep is its two colour kernels: per update, their sums
    if "sparse0" in agg and "sparse1" in agg:
        tot = {c: sum(sum(agg[k][c]) / len(agg[k][c]) for k in ("sparse0", "sparse1") if agg[k].get(c))
               for c in ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_VALU2",
                         "SQ_INSTS_VALU_TRANS_F32", "GRBM_GUI_ACTIVE")}
        act, act2 = tot["SQ_ACTIVE_INST_VALU"], tot["SQ_ACTIVE_INST_VALU2"]
        quads = tot["GRBM_GUI_ACTIVE"] / N_XCD / 4.0
        rate = act / (N_SIMD * quads) if quads else float("nan")
        n = min(len(agg["sparse0"].get("SQ_INSTS_VALU", [])), len(agg["sparse1"].get("SQ_INSTS_VALU", [])))
        out.append("| sparse0 + sparse1 (one sweep) | %d | %.4g | %.3f | %.3f | %.3f | %.3f | %.1f | %.2f |" % (
            n, tot["SQ_INSTS_VALU"], rate, rate, rate / 2.0, act2 / act if act else 0.0,
            act * 64.0 / updates, tot["SQ_INSTS_VALU_TRANS_F32"] * 64.0 / updates))
    return "\n".join(out)


def traffic(fetch_dir, write_dir, copy_mib):
    """Per inference sweep: the fused kernel's dispatch, or the two colour kernels of the
    compacted path added."""
    res = {}
    for d, ctr in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        kinds, probe = collections.defaultdict(list), []
        rows = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
        first = _probe_dispatch(rows)
        for r in rows:
            if r["Counter_Name"] != ctr:
                continue
            if _is_copy(r):
                if int(r["Dispatch_Id"]) == first:
                    probe.append(float(r["Counter_Value"]))
            else:
                k = _infer_sweep_kind(r["Kernel_Name"])
                if k:
                    kinds[k].append(float(r["Counter_Value"]))
        if not kinds or len(probe) != 1:
            raise SystemExit("%s: %d sweep kernels, %d copy probes" % (d, len(kinds), len(probe)))
        # the path the run swept with is the one with the most dispatches (an autotuner at load
        # also launches the other paths' kernels a few times); the compacted path's sweep is
        # its two colour kernels
        main = max(kinds, key=lambda k: len(kinds[k]))
        keep = ["sparse0", "sparse1"] if main.startswith("sparse") else [main]
        kinds = {k: v for k, v in kinds.items() if k in keep}
        factor = copy_mib * 1024.0 / probe[0]          # true KiB per counted KiB
        kib = sum(sum(v) / len(v) for v in kinds.values())
        res[ctr] = {"kib_per_sweep": kib, "factor": factor, "kernels": sorted(kinds),
                    "dispatches": sum(len(v) for v in kinds.values()), "bytes": kib * 1024.0 * factor}
    return {"fetch": res["FETCH_SIZE"], "write": res["WRITE_SIZE"],
            "bytes_per_launch": res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]}


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(stats(argv[1]))
    elif len(argv) >= 2 and argv[0] == "pmc":
        print(pmc(argv[1:]))
    elif len(argv) >= 3 and argv[0] == "valu":
        print(valu(argv[1], float(argv[2])))
    elif len(argv) >= 5 and argv[0] == "traffic":
        key, copy_mib, fdir, wdir = argv[1], float(argv[2]), argv[3], argv[4]
        entry = traffic(fdir, wdir, copy_mib)
        if len(argv) >= 6:
            out = argv[5]
            doc = {}
            if os.path.exists(out):
                doc = json.load(open(out))
            sha = kernel_source_sha()
            if doc.get("kernel_source_sha") != sha:
                doc = {"kernel_source_sha": sha, "entries": {}}
            doc["entries"][key] = entry
            with open(out, "w") as f:
                json.dump(doc, f, indent=1, sort_keys=True)
                f.write("\n")
        print(json.dumps({key: entry}, indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
