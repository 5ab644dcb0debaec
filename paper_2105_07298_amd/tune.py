"""Offline autotuner for the tile configurations (the paper tunes its block size by
sweeping TB, Sect. 3.2 and 4.1; here the sweep is automated and its result is a
table compiled into the library).

Run on the GPU:  python -m paper_2105_07298_amd.tune --out DIR
It times, with HIP events on the current stream,
  * fw_apsp for every compiled (block, tile_m, tile_n, variant), under each round schedule
    that applies to it (serial; lookahead; pairs), at one representative n per size
    range, for float32/float64 with and without the path matrix, on complete
    graphs with weights uniform in (0, 1), and for binary16 on complete graphs
    with integer weights in [1, 1000] (its exact range);
  * fw_apsp_batched on batches of equal-size graphs (weights in [1, 10],
    density 0.5) in 32 x 32 tiles and in 64 x 64 tiles, at the top size
    n = 32 (c + 1) of every size class c (n in (32c, 32c + 32]) up to 768
    vertices; a class takes 64 x 64 tiles when they were faster there (both
    tilings pad every n of a class to the same size as its top one), and every
    class above the timed range takes them (their padding costs at most
    (1 + 32/768)^3 = 1.13 times the work there, against the 1.4 to 1.7 times
    that 64 x 64 tiles gained at 384 to 512 vertices when this was written).
and writes DIR/tune_table.json (every timing) and DIR/tune_table.inc (the
table the library compiles; copy it to csrc/ and rebuild).  Tuning never changes
results: the tests check that every configuration gives the same D and P.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# size ranges [lo, hi) of the table and the n timed for each
BUCKETS = [(0, 384, 256), (384, 768, 512), (768, 1536, 1024), (1536, 3072, 2048), (3072, 6144, 4096),
           (6144, 12288, 8192), (12288, 1 << 40, 16384)]
BATCHED_CLASSES = 24  # size classes timed: n up to 32 * 24 = 768


def _timeit(fn, torch, reps, warmup=1):
    for _ in range(warmup):
        fn()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def tune_apsp(fw, torch, log, dtypes=("f32", "f64", "f16")):
    import numpy as np
    import workloads
    table = []
    codes = {"f32": fw.FW_F32, "f64": fw.FW_F64, "f16": fw.FW_F16}
    for dt in dtypes:
        for lo, hi, n in BUCKETS:
            if dt == "f16":
                W = torch.from_numpy(workloads.int_graph(n, 1.0, 1000, seed=2).astype(np.float16)).cuda()
            else:
                npdt = np.float32 if dt == "f32" else np.float64
                W = torch.from_numpy(workloads.unit_complete(n, dtype=npdt, seed=2)).cuda()
            D = torch.empty_like(W)
            for path in (False, True):
                P = torch.empty((n, n), dtype=torch.int32, device=W.device) if path else None
                best = None
                cands = [(b, tm, tn, var, sch) for b, tm, tn, var in fw.fw_list_configs(codes[dt])
                    for sch in (fw.FW_SCHED_SERIAL, fw.FW_SCHED_LOOKAHEAD, fw.FW_SCHED_PAIRS, fw.FW_SCHED_PAIRS_LOOKAHEAD)
                    if sch == fw.FW_SCHED_SERIAL or (sch == fw.FW_SCHED_LOOKAHEAD and fw.lookahead_applies(b, tm, tn, n))
                    or (sch == fw.FW_SCHED_PAIRS and fw.pairs_applies(b, tm, tn, var, n))
                    or (sch == fw.FW_SCHED_PAIRS_LOOKAHEAD and fw.pairs_lookahead_applies(b, tm, tn, var, n))]
                for block, tm, tn, var, sch in cands:
                    def run():
                        D.copy_(W)
                        fw.apsp_(D, P, block=block, tile_m=tm, tile_n=tn, variant=var, schedule=sch)
                    reps = 2 if n >= 8192 else 5
                    ms = _timeit(run, torch, reps)
                    log.append({"kind": "apsp", "dtype": dt, "path": path, "n": n, "block": block, "tile_m": tm,
                                "tile_n": tn, "variant": var, "schedule": sch, "ms": round(ms, 4)})
                    print(f"apsp {dt} path={path} n={n} block={block} tile={tm}x{tn} variant={var} "
                          f"schedule={sch}: {ms:.3f} ms", flush=True)
                    if best is None or ms < best[0]:
                        best = (ms, block, tm, tn, var, sch)
                table.append({"dtype": codes[dt], "path": path, "n_lo": lo, "n_hi": hi, "block": best[1],
                              "tile_m": best[2], "tile_n": best[3], "variant": best[4], "schedule": best[5]})
            del W, D
            torch.cuda.empty_cache()
    return table


def tune_batched(fw, torch, log):
    """tile64: bit c set when 64 x 64 tiles solve graphs of size class c
    (n in (32c, 32c + 32]) faster than 32 x 32 tiles; classes above the timed
    range are set."""
    import numpy as np
    import workloads
    table = []
    for dt in ("f32", "f64"):
        npdt = np.float32 if dt == "f32" else np.float64
        for path in (False, True):
            mask = ((1 << 64) - 1) & ~((1 << BATCHED_CLASSES) - 1)
            for c in range(BATCHED_CLASSES):
                n = 32 * (c + 1)
                count = int(max(64, min(4096, 2.0e9 / n ** 3 * 64)))
                g = workloads.graph(11, n, 0.5, workloads.W_ONE_TEN, 0, npdt)
                W = torch.from_numpy(np.tile(g.ravel(), count)).cuda()
                ns = np.full(count, n, dtype=np.int32)
                offs = np.arange(count, dtype=np.int64) * n * n
                D = torch.empty_like(W)
                P = torch.empty(W.shape, dtype=torch.int32, device=W.device) if path else None
                res = {}
                for split, label in ((1 << 20, 32), (0, 64)):
                    def run():
                        D.copy_(W)
                        fw.apsp_batched_(D, ns, offs, P, small_max_n=split)
                    res[label] = _timeit(run, torch, 3)
                    log.append({"kind": "batched", "dtype": dt, "path": path, "n": n, "tile": label,
                                "count": count, "ms": round(res[label], 4)})
                print(f"batched {dt} path={path} n={n} x{count}: 32-tiles {res[32]:.3f} ms, "
                      f"64-tiles {res[64]:.3f} ms", flush=True)
                if res[64] < res[32]:
                    mask |= 1 << c
                del W, D, P
            table.append({"dtype": fw.FW_F64 if dt == "f64" else fw.FW_F32, "path": path,
                          "tile64": f"0x{mask:016X}"})
    return table


def write_inc(path, apsp_table, batched_table, arch):
    lines = [
        "// Tile configuration table.  Generated by paper_2105_07298_amd/tune.py from",
        f"// timings on {arch} (do not edit by hand; rerun the tuner instead).",
        "// fw_apsp:          {dtype, path, n_lo, n_hi, block, tile_m, tile_n, variant, schedule}  n_lo <= n < n_hi",
        "// fw_apsp_batched:  {dtype, path, tile64}  bit c of tile64: 64 x 64 tiles for n in (32c, 32c + 32]",
        "//                   dtype: 0 float32, 1 float64, 2 binary16",
        f"// generated {time.strftime('%Y-%m-%d')}",
        "static const TuneEntry kTuneApsp[] = {",
    ]
    for t in apsp_table:
        hi = "1LL << 40" if t["n_hi"] >= (1 << 40) else str(t["n_hi"])
        lines.append(f"    {{{int(t['dtype'])}, {int(t['path'])}, {t['n_lo']}, {hi}, {t['block']}, {t['tile_m']}, "
                     f"{t['tile_n']}, {t['variant']}, {t['schedule']}}},")
    lines.append("};")
    lines.append("static const TuneBatchedEntry kTuneBatched[] = {")
    for t in batched_table:
        lines.append(f"    {{{int(t['dtype'])}, {int(t['path'])}, {t['tile64']}ull}},")
    lines.append("};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", required=True)
    ap.add_argument("--skip-apsp", action="store_true")
    ap.add_argument("--dtypes", default="f32,f64,f16", help="element types to time for fw_apsp")
    ap.add_argument("--keep", default="", help="tune_table.json whose rows are kept for the element types "
                    "not timed (and whose batched rows are kept with --skip-batched)")
    ap.add_argument("--skip-batched", action="store_true")
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import torch
    import paper_2105_07298_amd as fw
    fw.lib()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    os.makedirs(args.out, exist_ok=True)
    log = []
    dtypes = tuple(d for d in args.dtypes.split(",") if d)
    apsp_table = [] if args.skip_apsp else tune_apsp(fw, torch, log, dtypes)
    batched_table = [] if args.skip_batched else tune_batched(fw, torch, log)
    if args.keep:
        with open(args.keep) as f:
            old = json.load(f)
        codes = {"f32": fw.FW_F32, "f64": fw.FW_F64, "f16": fw.FW_F16}
        timed = {codes[d] for d in dtypes} if not args.skip_apsp else set()
        apsp_table = [t for t in old["apsp"] if t["dtype"] not in timed] + apsp_table
        apsp_table.sort(key=lambda t: (t["dtype"], t["n_lo"], t["path"]))
        if args.skip_batched:
            batched_table = old["batched"]
        log = [t for t in old["timings"]
               if not ((t["kind"] == "apsp" and codes[t["dtype"]] in timed)
                       or (t["kind"] == "batched" and not args.skip_batched))] + log
    with open(os.path.join(args.out, "tune_table.json"), "w") as f:
        json.dump({"arch": arch, "apsp": apsp_table, "batched": batched_table, "timings": log}, f, indent=1)
    write_inc(os.path.join(args.out, "tune_table.inc"), apsp_table, batched_table, arch)
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
