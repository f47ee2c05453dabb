"""Summarise rocprofv3 SQLite output (kernel trace and FETCH_SIZE / WRITE_SIZE
counter passes) as text.

    python -m paper_2606_05297_amd.rocprof_summary --trace T.db [--fetch F.db] [--write W.db]
           [--copy-bytes N | --fetch-factor F --write-factor W] [--json out.json]
           [--traffic-out traffic.json] [--split]

--split adds the time split of the trace: its span, the time some kernel runs
(the union of the kernel intervals), the idle time, the median gap between
consecutive kernels, and the kernel time per stage of the ADAPT step (SPLIT).

Counter scaling: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are converted to
bytes with the factor that makes the plain device copy kernel
(__amd_rocclr_copyBuffer, reading and writing N bytes) read exactly N bytes,
resp. write exactly N bytes; runs without such a copy take the factors
measured in a run that has one.

--traffic-out writes, per kernel family (the groups the library's own
profiling counters use), the HBM bytes (fetch + write) of one library call of
the family (summed over the kernels one call dispatches) and a hash of the
family's sources, so that a reader can tell whether the kernels changed since
the counters were taken.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sqlite3
from collections import defaultdict

COPY = "__amd_rocclr_copyBuffer"
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# kernel family -> (variants, source files the family is built from).  One
# library call of a family runs one dispatch of each stage of a variant (a
# stage lists the kernel base names that can fill it); its bytes per call are
# the sum over the stages of the mean bytes per dispatch.  The first variant
# whose stages all appear in the counter runs is used.
FAMILIES = {
    "apply_h": (((("k_h8_col",), ("k_h8_row",)), (("k_apply_h", "k_apply_h_lanes8"),)),
                ("stencil2.hip", "kernels_h.hip", "stencil_kernels.h", "device_common.h")),
    "pool_grads": (((("k_pool8_row",), ("k_pool8_col",)), (("k_pool",),)),
                   ("stencil2.hip", "kernels_pool.hip", "stencil_kernels.h", "device_common.h")),
    "score": (((("k_h8_col",), ("k_h8_row_score",), ("k_pool8_col",)),), ("stencil2.hip", "device_common.h")),
    "gate2": (((("k_gate2", "k_gate2_m0", "k_gate2_m0p", "k_gate2_half"),),),
              ("gate_kernels.h", "kernels_gate.hip", "gate_half.hip", "device_common.h")),
    "gate2_adjoint": (((("k_gate2_adj", "k_gate2_adj_m0", "k_gate2_adj_m0p", "k_gate2_adj_half"),),),
                      ("gate_kernels.h", "kernels_gate.hip", "gate_half.hip", "device_common.h")),
    "diag_gate": (((("k_diag", "k_diag_adj"),),), ("gate_kernels.h", "kernels_gate.hip", "device_common.h")),
    "apply_h_real": (((("k_h8_col_r",), ("k_h8_row_r",)),), ("stencil2.hip", "device_common.h")),
    "gate2_real": (((("k_rgate2", "k_rgate2_m0p", "k_rgate2_half"),),),
                   ("gate_real.hip", "gate_real_groups.h", "gate_kernels.h", "device_common.h")),
    "gate2_adjoint_real": (((("k_rgate2_adj", "k_rgate2_adj_m0p", "k_rgate2_adj_half"),),),
                           ("gate_real.hip", "gate_real_groups.h", "gate_kernels.h", "device_common.h")),
    "gate2_real_fused": (((("k_rfuse",),),),
                         ("gate_real_fuse.hip", "gate_real_groups.h", "gate_kernels.h", "device_common.h")),
    "gate2_adjoint_real_fused": (((("k_rfuse_adj",),),),
                                 ("gate_real_fuse.hip", "gate_real_groups.h", "gate_kernels.h", "device_common.h")),
    "real_convert": (((("k_real_to_complex", "k_complex_to_real"),),), ("gate_real.hip", "device_common.h")),
}


# stages of the ADAPT step for --split: (label, kernel base names); the last
# entry takes every other kernel.
SPLIT = [
    ("fused reverse runs on real states", ("k_rfuse_adj",)),
    ("fused forward runs on real states", ("k_rfuse",)),
    ("reverse step on real states (single gates)", ("k_rgate2_adj", "k_rgate2_adj_m0p", "k_rgate2_adj_half")),
    ("forward gates on real states (single gates)", ("k_rgate2", "k_rgate2_m0p", "k_rgate2_half")),
    ("real <-> complex conversion", ("k_real_to_complex", "k_complex_to_real")),
    ("reverse step, top pair (6,7) of the parity-halved layout", ("k_gate2_adj_half",)),
    ("reverse step, mode-0 pair (0,1)", ("k_gate2_adj_m0p", "k_gate2_adj_m0")),
    ("reverse step, other pairs", ("k_gate2_adj",)),
    ("forward gates, top pair (6,7) of the parity-halved layout", ("k_gate2_half",)),
    ("forward gates, mode-0 pair (0,1)", ("k_gate2_m0p", "k_gate2_m0")),
    ("forward gates, other pairs", ("k_gate2",)),
    ("apply-H row pass", ("k_h8_row",)),
    ("column pass (apply-H and scoring)", ("k_h8_col",)),
    ("apply-H on real states (column + row pass)", ("k_h8_col_r", "k_h8_row_r")),
    ("scoring (fused row pass, column pool pass)", ("k_h8_row_score", "k_pool8_col", "k_pool8_row")),
    ("other kernels (reductions, copies, gate builds, sector conversion)", None),
]


def split(db):
    """Span, busy time (union of kernel intervals), idle time, median gap
    between consecutive kernels, and kernel time per SPLIT stage."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    if not rows:
        return
    busy, cur_s, cur_e, gaps = 0, rows[0][1], rows[0][2], []
    per = defaultdict(float)
    for n, st, en in rows:
        if st > cur_e:
            busy += cur_e - cur_s
            gaps.append(st - cur_e)
            cur_s, cur_e = st, en
        else:
            cur_e = max(cur_e, en)
        b = base_of(short(n))
        lab = next(lab for lab, names in SPLIT if names is None or b in names)
        per[lab] += en - st
    busy += cur_e - cur_s
    span = rows[-1][2] - rows[0][1]
    gaps.sort()
    med = gaps[len(gaps) // 2] / 1e3 if gaps else 0.0
    ktot = sum(per.values())
    print(f"{len(rows)} kernels over {span / 1e6:.1f} ms: some kernel runs for {busy / 1e6:.1f} ms, idle "
          f"{(span - busy) / 1e6:.1f} ms, median gap between consecutive kernels {med:.2f} us")
    for lab, _ in SPLIT:
        if per.get(lab):
            print(f"  {lab:66s} {per[lab] / 1e6:9.1f} ms  {100 * per[lab] / ktot:5.1f} %")


def source_sha(family: str) -> str:
    h = hashlib.sha256()
    for f in FAMILIES[family][1]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def base_of(kname: str) -> str:
    """Kernel base name; the real-state instantiations of the slab H passes
    (two reals per float2, one per float) get a name of their own."""
    b = kname.split("<")[0].split("::")[-1]
    if b == "k_h8_col" and "float, 2u" in kname:
        return "k_h8_col_r"
    if b == "k_h8_row" and re.search(r"k_h8_row<float\s*>", kname):
        return "k_h8_row_r"
    return b


def family_bytes(fam: str, per_kernel: dict):
    """Bytes per library call of family fam from per-kernel dispatch values
    (mean over the dispatches of each stage, summed over the stages), with the
    number of dispatches used; None when no variant is complete."""
    for stages in FAMILIES[fam][0]:
        total, n = 0.0, 0
        for stage in stages:
            vals = [v for k, vs in per_kernel.items() if base_of(k) in stage for v in vs]
            if not vals:
                break
            total += sum(vals) / len(vals)
            n += len(vals)
        else:
            return total, n
    return None


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    m = re.match(r"^(?:void )?([\w:]+(?:<[^()]*>)?)", name)
    return m.group(1) if m else name[:80]


def trace(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels").fetchall()
    agg = defaultdict(list)
    for n, d in rows:
        agg[short(n)].append(d)
    return agg


def counter(db, cname):
    """Per-kernel counter values; copy-kernel dispatches are kept only at the
    largest grid (the full-state copy of known size)."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, value, grid_size from counters_collection where counter_name = ?",
                       (cname,)).fetchall()
    gmax = max([g for n, v, g in rows if short(n) == COPY] or [0])
    agg = defaultdict(list)
    for n, v, g in rows:
        if short(n) == COPY and g != gmax:
            continue
        agg[short(n)].append(v)
    return agg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-bytes", type=float, default=0.0)
    ap.add_argument("--fetch-factor", type=float, default=None)
    ap.add_argument("--write-factor", type=float, default=None)
    ap.add_argument("--json")
    ap.add_argument("--traffic-out")
    ap.add_argument("--split", action="store_true")
    a = ap.parse_args()
    tr = trace(a.trace)
    fe = counter(a.fetch, "FETCH_SIZE") if a.fetch else {}
    wr = counter(a.write, "WRITE_SIZE") if a.write else {}
    ffac = wfac = None
    if a.copy_bytes and COPY in fe:
        ffac = a.copy_bytes / (1024.0 * sum(fe[COPY]) / len(fe[COPY]))
    if a.copy_bytes and COPY in wr:
        wfac = a.copy_bytes / (1024.0 * sum(wr[COPY]) / len(wr[COPY]))
    ffac = a.fetch_factor if a.fetch_factor is not None else ffac
    wfac = a.write_factor if a.write_factor is not None else wfac
    print(f"{'kernel':60s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'fetch_MB':>10s} {'write_MB':>10s}")
    out = {"fetch_factor": ffac, "write_factor": wfac, "kernels": {}}
    for k in sorted(tr, key=lambda k: -sum(tr[k])):
        d = tr[k]
        avg = sum(d) / len(d) / 1e3
        f = (sum(fe[k]) / len(fe[k]) * 1024.0 * (ffac or 1.0)) if k in fe else None
        w = (sum(wr[k]) / len(wr[k]) * 1024.0 * (wfac or 1.0)) if k in wr else None
        out["kernels"][k] = {"calls": len(d), "avg_us": avg, "total_ms": sum(d) / 1e6, "fetch_bytes": f,
                             "write_bytes": w}
        fs = f"{f / 1e6:10.1f}" if f is not None else f"{'-':>10s}"
        ws = f"{w / 1e6:10.1f}" if w is not None else f"{'-':>10s}"
        print(f"{k[:60]:60s} {len(d):6d} {avg:10.2f} {sum(d) / 1e6:10.3f} {fs} {ws}")
    if ffac or wfac:
        print(f"counter scale factors (copy kernel): fetch x{ffac}, write x{wfac}")
    if a.split:
        split(a.trace)
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(out, fh, indent=1)
    if a.traffic_out and fe and wr and ffac and wfac:
        fam = {}
        for f in FAMILIES:
            fb, wb = family_bytes(f, fe), family_bytes(f, wr)
            if fb and wb:
                fetch, write = 1024.0 * ffac * fb[0], 1024.0 * wfac * wb[0]
                fam[f] = {"hbm_bytes_per_launch": fetch + write, "fetch_bytes_per_launch": fetch,
                          "write_bytes_per_launch": write, "dispatches": fb[1], "source_sha": source_sha(f)}
                print(f"family {f:14s} dispatches {fb[1]:5d}  HBM bytes per call {(fetch + write) / 1e6:10.1f} MB")
        with open(a.traffic_out, "w") as fh:
            json.dump({"fetch_factor": ffac, "write_factor": wfac, "families": fam}, fh, indent=1)


if __name__ == "__main__":
    main()
