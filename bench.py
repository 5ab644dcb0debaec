#!/usr/bin/env python3
"""Benchmark of the blocked Floyd-Warshall APSP library on one MI355X.

Headline: GFLOPS = 2 n^3 / t (paper Sect. 4.2, Eq. 1) at n = 16384 in float32 with
the path matrix -- the full output of Algorithm 1 -- on a complete directed graph
with weights uniform in (0, 1).  One step = D <- W (device copy), P <- -1, and
all rounds of the blocked method: one whole fw_apsp call.  Inputs are resident in
HBM before the timed region.  Timing: W untimed warm-up steps, then K steps
between device synchronizations, timed with events on the stream the library
runs on; the paper averages 15 repetitions (Sect. 4.1).

Also reported:
  roofline      the last-phase kernel (the min-plus tile update, >98% of the
                work): algorithmic flops per launch / its mean launch duration
                (events around every launch during the timed steps) against the
                vector-ALU bound of its instruction mix.
  cpu_baseline  the CPU oracle (classic triple loop, float64) on the same
                matrix, a bounded prefix of its outer iterations, on all cores.
  secondary     float64, distances-only, and (when built) batched and backward
                figures on the same GPU.

Prints one JSON line.  --gpus above 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "APSP GFLOPS=2n³/t at n=16384 FP32/FP64; batched graphs/s; fwd+bwd vs fwd"

# Vector-ALU bound of the last-phase kernel, in 2-flop updates.  256 CUs x 4 SIMDs
# at 2.4 GHz; a SIMD retires 32 lanes/clk of v_add_f32 and 16 lanes/clk of
# v_min3_f32, v_add_f64 and v_min_f64.  float32 spends one v_add_f32 and half a
# v_min3_f32 per update (1/32 + 0.5/16 = 1/16 SIMD-clk per lane-update), float64
# one v_add_f64 and one v_min_f64 (1/8).  Hence 64 (float32) and 32 (float64)
# updates per CU per clock.  binary16 (FW_F16) updates two entries per packed
# instruction: two v_pk_add_f16 and one v_pk_minimum3_f16 (16 lanes/clk each)
# per 4 updates, 3/64 SIMD-clk per lane-update, 85.3 updates per CU per clock.
CU_CLK = 256 * 2.4e9
PEAK_TFLOPS = {"f32": CU_CLK * 64 * 2 / 1e12, "f64": CU_CLK * 32 * 2 / 1e12, "f16": CU_CLK * 256 / 3 * 2 / 1e12}
DT_CODE = {"f32": 0, "f64": 1, "f16": 2}
# The last-phase kernel's source: its file and the headers it includes (the
# measured traffic in TRAFFIC_FILE is valid for these exact sources only).
KERNEL_SRC = [os.path.join(ROOT, "paper_2105_07298_amd", "csrc", f)
              for f in ("fw_kernels.hip", "fw_internal.h", "fw_lex.h", "fw_tiles.h", "fw_device.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for src in KERNEL_SRC:
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def gflops(n, seconds):
    return 2.0 * n ** 3 / seconds / 1e9


class EnergyMeter:
    """GPU energy over a timed region: the device's accumulated energy counter
    (amdsmi), read before and after; socket power sampled every 20 ms alongside.
    Every field is None, with a reason, where the counters cannot be read."""

    def __init__(self, torch):
        self.handle, self.reason = None, ""
        try:
            import amdsmi
            self.smi = amdsmi
            amdsmi.amdsmi_init(amdsmi.AmdSmiInitFlags.INIT_AMD_GPUS)
            handles = amdsmi.amdsmi_get_processor_handles()
            if len(handles) == 1:
                self.handle = handles[0]
            else:  # pick the device torch uses by PCI bus
                props = torch.cuda.get_device_properties(torch.cuda.current_device())
                bus = getattr(props, "pci_bus_id", None)
                for h in handles:
                    bdf = amdsmi.amdsmi_get_gpu_device_bdf(h)
                    if bus is not None and int(bdf.split(":")[1], 16) == bus:
                        self.handle = h
                if self.handle is None:
                    self.reason = f"{len(handles)} GPUs visible to amdsmi and none matched the PCI bus"
        except Exception as e:  # no driver access, no library, ...
            self.reason = f"amdsmi unavailable: {e}"

    def _energy_uj(self):
        e = self.smi.amdsmi_get_energy_count(self.handle)
        return e["energy_accumulator"] * e["counter_resolution"]

    def _sample(self):
        while not self._stop.is_set():
            try:
                pw = self.smi.amdsmi_get_power_info(self.handle)
                v = pw.get("current_socket_power")
                if not isinstance(v, (int, float)) or v <= 0 or v > 10000:
                    v = pw.get("average_socket_power")
                if isinstance(v, (int, float)) and 0 < v < 10000:
                    self._samples.append(float(v))
            except Exception:
                pass
            self._stop.wait(0.02)

    def start(self):
        import threading
        if self.handle is None:
            return
        self._samples, self._stop = [], threading.Event()
        self._t0 = time.perf_counter()
        try:
            self._e0 = self._energy_uj()
        except Exception as e:
            self._e0, self.reason = None, f"energy counter unreadable: {e}"
        self._thr = threading.Thread(target=self._sample, daemon=True)
        self._thr.start()

    def stop(self, steps, flops_per_step):
        out = {"joules_per_step": None, "avg_power_w": None, "sampled_power_w": None, "gflops_per_w": None,
               "source": None, "reason": self.reason or None}
        if self.handle is None:
            return out
        sec = time.perf_counter() - self._t0
        self._stop.set()
        self._thr.join()
        if self._samples:
            out["sampled_power_w"] = round(sum(self._samples) / len(self._samples), 1)
        if self._e0 is not None:
            joules = (self._energy_uj() - self._e0) / 1e6
            if joules > 0:
                out.update({"joules_per_step": round(joules / steps, 3), "avg_power_w": round(joules / sec, 1),
                            "gflops_per_w": round(flops_per_step * steps / joules / 1e9, 2),
                            "source": "amdsmi energy accumulator over the timed steps", "reason": None})
                return out
        if out["sampled_power_w"]:
            out.update({"avg_power_w": out["sampled_power_w"],
                        "gflops_per_w": round(flops_per_step * steps / sec / 1e9 / out["sampled_power_w"], 2),
                        "source": "amdsmi socket power, sampled every 20 ms"})
        return out


def run_stats(step_ms):
    """mean / min / median of the per-step times (ms) of the timed runs."""
    import numpy as np
    a = np.asarray(step_ms, dtype=np.float64)
    return {"runs": int(a.size), "mean_ms": round(float(a.mean()), 4), "min_ms": round(float(a.min()), 4),
            "median_ms": round(float(np.median(a)), 4)}


def timed_steps(torch, step, steps, warmup):
    """W untimed warm-ups, then K steps between device synchronizations, each
    bracketed by events on the current stream.  Returns (seconds for all K, per-step ms)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return ev[0].elapsed_time(ev[steps]) / 1e3, per


def time_apsp(fw, torch, n, dtype, path, steps, warmup, prof=False, config=None, energy=None, prof_apart=False):
    """Mean seconds per fw_apsp step (D <- W, P <- -1, all rounds), the per-step
    times and last-phase stats.  config: (block, tile_m, tile_n, variant, schedule),
    default the tuned choice.  The last-phase stats come from events around every
    bulk launch of the timed steps; with prof_apart, from 3 more steps after them
    instead, so that the timed steps carry no event records (a few microseconds per
    launch, which matter at small n)."""
    import numpy as np
    import workloads
    block, tm, tn, var, sch = config or fw.fw_query_config(DT_CODE[dtype], n, path)
    if dtype == "f16":  # integer weights in [1, 1000]: every distance is exact in binary16
        Wd = torch.from_numpy(workloads.int_graph(n, 1.0, 1000, seed=2).astype(np.float16)).cuda()
    else:
        npdt = np.float32 if dtype == "f32" else np.float64
        Wd = torch.from_numpy(workloads.unit_complete(n, dtype=npdt, seed=2)).cuda()
    D = torch.empty_like(Wd)
    P = torch.empty((n, n), dtype=torch.int32, device=Wd.device) if path else None

    def step():
        D.copy_(Wd)
        fw.apsp_(D, P, block=block, tile_m=tm, tile_n=tn, variant=var, schedule=sch)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if prof and not prof_apart:
        fw.fw_prof_read(reset=True)
        fw.fw_prof_enable(True)
    if energy is not None:
        energy.start()
    total, per = timed_steps(torch, step, steps, 0)
    if energy is not None:
        energy.result = energy.stop(steps, 2.0 * n ** 3)
    sec = total / steps
    stats = None
    if prof and prof_apart:
        fw.fw_prof_read(reset=True)
        fw.fw_prof_enable(True)
        timed_steps(torch, step, 3, 0)
    if prof:
        fw.fw_prof_enable(False)
        cnt, tot_ms, upd = fw.fw_prof_read(reset=True)
        stats = {"launches": cnt, "mean_ms": tot_ms / max(cnt, 1), "block": block, "tile": [tm, tn],
                 "variant": var, "schedule": sch, "updates_per_launch": upd / max(cnt, 1)}
    del Wd, D, P
    torch.cuda.empty_cache()
    return sec, stats, per


def time_large(fw, torch, dtype, runs, warmup, meter=None):
    """The large single graph: n = 65536, edge probability 0.1, integer weights in
    [1, 100], distances and path matrix.  Before every call the input is generated
    on the device (the generator's device twin) straight into D, outside the
    timing; each call is timed by events on the current stream, and the energy
    counter is read around each timed call alone."""
    import workloads
    n = 65536
    tdt = torch.float32 if dtype == "f32" else torch.float64
    D = torch.empty((n, n), dtype=tdt, device="cuda")
    P = torch.empty((n, n), dtype=torch.int32, device="cuda")
    per, runs_e = [], []
    for r in range(warmup + runs):
        workloads.rows_dev(3, n, 0, n, 0.1, workloads.W_INT, 100, D)
        torch.cuda.synchronize()
        timed = r >= warmup
        if timed and meter is not None:
            meter.start()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fw.apsp_(D, P)
        e1.record()
        torch.cuda.synchronize()
        if timed:
            per.append(e0.elapsed_time(e1))
            if meter is not None:
                runs_e.append(meter.stop(1, 2.0 * n ** 3))
    del D, P
    torch.cuda.empty_cache()
    sec = sum(per) / len(per) / 1e3
    out = {"n": n, "dtype": dtype, "path": True, "gflops": round(gflops(n, sec), 2),
           "ms_per_call": round(sec * 1e3, 1), "timing": run_stats(per),
           "workload": "edge probability 0.1, integer weights in [1, 100], missing edges +inf",
           "note": f"{warmup} untimed call(s) first; input regenerated on the device before every call, "
                   "outside the timing"}
    if meter is not None:
        js = [e["joules_per_step"] for e in runs_e if e.get("joules_per_step")]
        if len(js) == len(runs_e) and js:
            j = sum(js) / len(js)
            out["energy"] = {"joules_per_call": round(j, 1), "avg_power_w": round(j / sec, 1),
                             "gflops_per_w": round(2.0 * n ** 3 / j / 1e9, 2), "dtype": dtype,
                             "source": "amdsmi energy accumulator around each timed call"}
        else:
            out["energy"] = dict(runs_e[-1] if runs_e else {}, dtype=dtype)
    return out


def time_batched(fw, torch, steps=15, warmup=2):
    """The batched workload: 10,000 graphs, n uniform in [16, 512], density uniform in
    [0.1, 1.0), float32 weights in [1, 10], path matrices, one persistent launch."""
    import numpy as np
    import workloads
    ns, off, W = workloads.batch_graphs(batch=10000, seed=4)
    Wd = torch.from_numpy(W).cuda()
    D = torch.empty_like(Wd)
    P = torch.empty(Wd.shape, dtype=torch.int32, device=Wd.device)
    offs = off[:-1].copy()

    def step():
        D.copy_(Wd)
        fw.apsp_batched_(D, ns, offs, P)

    total, per = timed_steps(torch, step, steps, warmup)
    sec = total / steps
    flops = 2.0 * float(np.sum(ns.astype(np.float64) ** 3))
    return {"graphs_per_s": round(ns.size / sec, 1), "ms_per_batch": round(sec * 1e3, 3),
            "gflops": round(flops / sec / 1e9, 2), "batch": int(ns.size), "n_range": [16, 512],
            "timing": run_stats(per)}


def time_ooc(fw, torch, n=32768, S=8192, path=False, runs=15, warmup=1):
    """Out of core: an n x n float32 complete graph (weights in (0,1)) in pinned host
    memory, through a device budget that holds super-blocks of edge S (n / S
    super-rounds).  Each call (transfers included) starts from the same weights,
    regenerated into the pinned buffer before it, outside the timing; `warmup`
    untimed calls come first (the first call of a process also pays one-time
    driver costs)."""
    import numpy as np
    import workloads
    nb = -(-n // S)
    blocks = 4 * S * S + 4 * S * nb * S
    budget = blocks * 4 + ((blocks + S * S) * 4 if path else 0)
    assert fw.fw_ooc_superblock(fw.FW_F32, n, path, budget) == S
    H = torch.empty((n, n), dtype=torch.float32, pin_memory=True)
    HP = torch.empty((n, n), dtype=torch.int32, pin_memory=True) if path else None
    Hn = H.numpy()
    times = []
    for r in range(warmup + runs):
        for i0 in range(0, n, 4096):  # the generator writes straight into the pinned rows
            i1 = min(n, i0 + 4096)
            workloads.rows(2, n, i0, i1, 1.0, workloads.W_UNIT_OPEN, 0, np.float32, 0, Hn[i0:i1])
        torch.cuda.synchronize()
        t = time.perf_counter()
        fw.apsp_ooc_(H, HP, budget)
        if r >= warmup:
            times.append(time.perf_counter() - t)
    sec = sum(times) / len(times)
    return {"n": n, "superblock": S, "device_bytes": budget, "seconds": round(sec, 3),
            "gflops": round(gflops(n, sec), 2), "dtype": "f32", "path": path,
            "timing": run_stats([t * 1e3 for t in times]),
            "warmup": warmup, "note": "matrix in pinned host memory; host-to-device and device-to-host transfers included"}


def time_fwd_bwd(fw, torch, steps=15, warmup=2):
    """Forward (D and P) and forward + backward (dL/dW for G ~ N(0,1)): n = 2048 complete
    graph with float32 weights in [1, 2), and a batch of 256 such graphs at n = 128."""
    import numpy as np
    import workloads

    def measure(W, G):
        Wd = torch.from_numpy(W).cuda()
        Gd = torch.from_numpy(G).cuda()

        def fwd():
            return fw._forward(Wd)

        def fwd_bwd():
            D, P = fw._forward(Wd)
            return fw.apsp_backward(D, P, Gd)

        D0, P0 = fw._forward(Wd)

        def bwd():
            return fw.apsp_backward(D0, P0, Gd)

        res = {}
        for name, fn in (("fwd", fwd), ("fwd_bwd", fwd_bwd), ("bwd", bwd)):
            total, per = timed_steps(torch, fn, steps, warmup)
            res[name + "_ms"] = round(total * 1e3 / steps, 3)
            res[name + "_timing"] = run_stats(per)
        res["ratio"] = round(res["fwd_bwd_ms"] / res["fwd_ms"], 3)
        return res

    W, G = workloads.grad_graph(n=2048, seed=5)
    single = measure(W, G)
    Ws = np.stack([workloads.grad_graph(n=128, seed=5, g=b)[0] for b in range(256)])
    Gs = np.stack([workloads.grad_graph(n=128, seed=5, g=b)[1] for b in range(256)])
    batch = measure(Ws, Gs)
    # The complete graph with weights in [1, 2) has D = W (every shortest path is its
    # direct edge), so its backward is a one-level scatter.  The same weights at edge
    # density 0.05 give multi-hop shortest paths and deep subtrees.
    Wsp, Gsp = workloads.grad_graph(n=2048, seed=5, p=0.05)
    sparse = measure(Wsp, Gsp)
    return {"n2048": single, "batch256_n128": batch,
            "n2048_density0.05": dict(sparse, note="non-degenerate: multi-hop shortest paths")}


def roofline(n, dtype, stats, path=True):
    block = stats["block"]
    upd = stats["updates_per_launch"]  # algorithmic min-plus updates per timed last-phase launch
    achieved = 2.0 * upd / (stats["mean_ms"] / 1e3) / 1e12
    peak = PEAK_TFLOPS[dtype]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        key = f"{dtype}_n{n}_{'path' if path else 'dist'}"
        if t.get("kernel_hash") == kernel_hash() and key in t:
            traffic = t[key]["bytes_per_launch"]
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic,
            "kernel": ("k_phase4w (wave-row min-plus tile update)" if stats["variant"] == 2
                       else "k_phase4 (LDS-panel min-plus tile update"
                       + (", fused pair of rounds)" if stats["schedule"] in (3, 4) else ")")),
            "schedule": {1: "serial", 2: "lookahead", 3: "pairs", 4: "pairs with lookahead"}.get(stats["schedule"],
                                                                                              stats["schedule"]),
            "tile": stats["tile"], "block": block, "launches": stats["launches"],
            "mean_launch_ms": round(stats["mean_ms"], 4), "flops_per_launch": 2 * upd}


def cpu_baseline(n, budget_s=15.0):
    """Oracle (float64 classic loop) on the same n x n matrix: a prefix of its outer
    iterations on all host cores, scaled to GFLOPS (each iteration is n^2 updates)."""
    import numpy as np
    import oracle
    import workloads
    W = workloads.unit_complete(n, dtype=np.float32, seed=2)
    D = W.astype(np.float64)
    del W
    P = np.full((n, n), -1, dtype=np.int32)
    cores = oracle.max_threads()
    k = 4
    oracle.fw_steps(D, P, 0, k)  # first iterations untimed (page-in of the matrix)
    # then chunks of 16 outer iterations until the budget is spent
    t = time.perf_counter()
    k2 = k
    while k2 < n and time.perf_counter() - t < budget_s:
        k3 = min(n, k2 + 16)
        oracle.fw_steps(D, P, k2, k3)
        k2 = k3
    dt = time.perf_counter() - t
    total_k = k2 - k
    g = 2.0 * n * n * total_k / dt / 1e9
    return {"value": round(g, 3), "unit": "GFLOPS", "cores": cores, "kind": "oracle",
            "sample": f"outer iterations {k}..{k2 - 1} of {n} of the float64 classic loop on the same "
                      f"n={n} matrix ({dt:.1f} s, {total_k * n * n:.3e} updates)",
            "extrapolated_full_run_s": round(dt / total_k * n, 1)}


def host_cpu():
    """CPU model and logical CPU count of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "sched_affinity": len(os.sched_getaffinity(0))}


class BackgroundOracle:
    """A single-thread oracle run in a Python thread (the C call releases the GIL),
    so that it overlaps GPU timing that needs only the launching thread."""

    def __init__(self, fn):
        import threading
        self.result = None
        self.t = threading.Thread(target=self._run, args=(fn,), daemon=True)
        self.t.start()

    def _run(self, fn):
        t = time.perf_counter()
        fn()
        self.result = time.perf_counter() - t

    def join(self):
        self.t.join()
        return self.result


def oracle_c2_4096_single():
    import numpy as np
    import oracle
    import workloads
    W = workloads.unit_complete(4096, dtype=np.float32, seed=2)
    return lambda: oracle.fw(W, exact=False, threads=1)


def oracle_timings(fw, torch, gpu_secondary, single_thread_s=None, runs=15):
    """The oracle timed fully on the small workloads, all host cores (and one thread
    where stated), beside the GPU figure for the same input:
      C1  n = 512, edge probability 0.5, integer weights in [1, 1000] (int64 loop);
      C2  n = 4096 complete graph, weights in (0, 1) (float64 loop);
      C4  the 10,000-graph batch (float64 loop per graph, graphs spread over the
          cores, one thread each);
      C5  n = 2048 complete graph, weights in [1, 2): forward (float64 loop) and the
          path-walk backward (serial), and the 256 x 128 batch likewise."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    import workloads
    cores = oracle.max_threads()
    out = {"cores": cores}

    def gpu_ms(W, path=True):
        Wd = torch.from_numpy(W).cuda()
        D = torch.empty_like(Wd)
        P = torch.empty(W.shape, dtype=torch.int32, device="cuda") if path else None

        def step():
            D.copy_(Wd)
            fw.apsp_(D, P)
        total, per = timed_steps(torch, step, runs, 2)
        return run_stats(per)

    W1 = workloads.int_graph(n=512, p=0.5, wmax=1000, seed=1)
    g1 = gpu_ms(W1)
    t = time.perf_counter()
    oracle.fw(W1)
    a = time.perf_counter() - t
    t = time.perf_counter()
    oracle.fw(W1, threads=1)
    b = time.perf_counter() - t
    out["C1_n512"] = {"oracle_s_all_cores": round(a, 4), "oracle_s_1_thread": round(b, 4), "gpu": g1,
                      "speedup_vs_all_cores": round(a * 1e3 / g1["mean_ms"], 1)}

    W2 = workloads.unit_complete(4096, dtype=np.float32, seed=2)
    g2 = gpu_ms(W2)
    t = time.perf_counter()
    oracle.fw(W2, exact=False)
    a = time.perf_counter() - t
    out["C2_n4096"] = {"oracle_s_all_cores": round(a, 3), "oracle_gflops_all_cores": round(gflops(4096, a), 2),
                       "oracle_s_1_thread": round(single_thread_s, 3) if single_thread_s else None,
                       "oracle_gflops_1_thread": round(gflops(4096, single_thread_s), 3) if single_thread_s else None,
                       "gpu": g2, "gpu_gflops": round(gflops(4096, g2["mean_ms"] / 1e3), 1),
                       "speedup_vs_all_cores": round(a * 1e3 / g2["mean_ms"], 1)}

    ns, off, W4 = workloads.batch_graphs(batch=10000, seed=4)
    graphs = [W4[off[b]:off[b + 1]].reshape(int(ns[b]), int(ns[b])) for b in range(ns.size)]
    order = np.argsort(-ns)  # largest first, as the GPU queue
    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(lambda b: oracle.fw(graphs[b], exact=False, threads=1), order))
    a = time.perf_counter() - t
    gb = (gpu_secondary or {}).get("batched", {})
    out["C4_batch10000"] = {"oracle_s_all_cores": round(a, 2), "oracle_graphs_per_s": round(ns.size / a, 1),
                            "gpu_ms": gb.get("ms_per_batch"), "gpu_graphs_per_s": gb.get("graphs_per_s"),
                            "speedup_vs_all_cores": round(a * 1e3 / gb["ms_per_batch"], 1) if gb else None}

    W5, G5 = workloads.grad_graph(n=2048, seed=5)
    t = time.perf_counter()
    D5, P5 = oracle.fw(W5, exact=False)
    a = time.perf_counter() - t
    t = time.perf_counter()
    oracle.backward_pathwalk(D5, P5, G5.astype(np.float64))
    b = time.perf_counter() - t
    Ws = [workloads.grad_graph(n=128, seed=5, g=g) for g in range(256)]
    t = time.perf_counter()
    res = [oracle.fw(w, exact=False) for w, _ in Ws]
    c = time.perf_counter() - t
    t = time.perf_counter()
    for (D, P), (_, G) in zip(res, Ws):
        oracle.backward_pathwalk(D, P, G.astype(np.float64))
    d = time.perf_counter() - t
    fb = (gpu_secondary or {}).get("fwd_bwd", {})
    out["C5"] = {"n2048": {"oracle_fwd_s": round(a, 3), "oracle_bwd_s": round(b, 3),
                           "gpu_fwd_ms": fb.get("n2048", {}).get("fwd_ms"),
                           "gpu_fwd_bwd_ms": fb.get("n2048", {}).get("fwd_bwd_ms")},
                 "batch256_n128": {"oracle_fwd_s": round(c, 3), "oracle_bwd_s": round(d, 3),
                                   "gpu_fwd_ms": fb.get("batch256_n128", {}).get("fwd_ms"),
                                   "gpu_fwd_bwd_ms": fb.get("batch256_n128", {}).get("fwd_bwd_ms")},
                 "note": "oracle forward on all cores, path-walk backward serial"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sec-steps", type=int, default=15, help="timed runs of every secondary figure")
    ap.add_argument("--no-oracle-timings", action="store_true",
                    help="skip the full oracle runs on the small workloads")
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--dtype", choices=["f32", "f64", "f16"], default="f32")
    ap.add_argument("--no-path", action="store_true", help="distances only (P = NULL)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-energy", action="store_true", help="skip the amdsmi energy reading")
    ap.add_argument("--config", default="", help="block,tile_m,tile_n,variant,schedule instead of the tuned choice")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the n = 65536 secondary figures")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched workload (10,000 graphs) and print its line")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, one device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py: --gpus {args.gpus} requested, but this library runs on one GPU; "
              "multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2105_07298_amd as fw
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    fw.lib()

    def calib_copy(out):
        if args.calib_copy_mib:
            nb = args.calib_copy_mib * (1 << 20)
            a = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            a.fill_(1.0)
            torch.cuda.synchronize()
            b.copy_(a)
            torch.cuda.synchronize()
            out["calib_copy_bytes"] = nb
        return out

    if args.batched_only:
        print("[bench] batched 10,000 graphs", file=sys.stderr, flush=True)
        r = time_batched(fw, torch, steps=args.steps, warmup=args.warmup)
        print(json.dumps(calib_copy({"metric": "batched APSP graphs/s", "value": r["graphs_per_s"], "unit": "graphs/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_batch"],
                          "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "10,000 graphs, n uniform in [16, 512], density uniform in "
                                                 "[0.1, 1.0), weights uniform real in [1, 10], path matrices"},
                          "gflops": r["gflops"]})), flush=True)
        return

    path = not args.no_path
    print(f"[bench] n={args.n} {args.dtype} path={path} warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)
    config = tuple(int(x) for x in args.config.split(",")) if args.config else None
    meter = None if args.no_energy else EnergyMeter(torch)
    sec, stats, per = time_apsp(fw, torch, args.n, args.dtype, path, args.steps, args.warmup, prof=True,
                                config=config, energy=meter)
    value = gflops(args.n, sec)
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GFLOPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"complete directed graph n={args.n}, "
                               + ("integer weights in [1, 1000], binary16, " if args.dtype == "f16" else
                                  f"weights uniform real in (0,1), {'float32' if args.dtype == 'f32' else 'float64'}, ")
                               + ("distances + path matrix" if path else "distances only"),
                   "n": args.n, "path": path, "block": stats["block"], "tile": stats["tile"],
                   "parallelism": "single GPU"},
        "timing": run_stats(per),
        "roofline": roofline(args.n, args.dtype, stats, path),
        "energy": meter.result if meter is not None else None,
    }
    calib_copy(out)
    single = None
    if not args.no_cpu_baseline and not args.no_oracle_timings:
        print("[bench] oracle n=4096 on one thread, in the background", file=sys.stderr, flush=True)
        single = BackgroundOracle(oracle_c2_4096_single())
    sec_out = None
    if not args.no_secondary:
        sec_out = {}
        K, Wu = args.sec_steps, args.warmup
        for dt_, pth in (("f64", True), ("f32", False), ("f64", False), ("f16", True), ("f16", False)):
            if dt_ == args.dtype and pth == path:
                continue
            print(f"[bench] secondary n={args.n} {dt_} path={pth}", file=sys.stderr, flush=True)
            m2 = EnergyMeter(torch) if (dt_ == "f64" and pth and not args.no_energy) else None
            s, st, p2 = time_apsp(fw, torch, args.n, dt_, pth, K, Wu, prof=True, energy=m2, prof_apart=True)
            key = f"{dt_}_{'path' if pth else 'dist'}"
            sec_out[key] = {"gflops": round(gflops(args.n, s), 2), "ms_per_step": round(s * 1e3, 2),
                            "timing": run_stats(p2), "roofline_frac": roofline(args.n, dt_, st, pth)["frac"]}
            if m2 is not None:
                sec_out[key]["energy"] = dict(m2.result, dtype="f64")
            if dt_ == "f16":
                sec_out[key]["workload"] = "complete graph, integer weights in [1, 1000] (exact in binary16)"
        for n2 in (4096, 8192):
            for dt_ in ("f32", "f64"):
                print(f"[bench] secondary n={n2} {dt_} path=True", file=sys.stderr, flush=True)
                s, st, p2 = time_apsp(fw, torch, n2, dt_, True, K, Wu, prof=True, prof_apart=True)
                sec_out[f"{dt_}_path_n{n2}"] = {"gflops": round(gflops(n2, s), 2), "ms_per_step": round(s * 1e3, 3),
                                                "timing": run_stats(p2),
                                                "roofline_frac": roofline(n2, dt_, st, True)["frac"]}
        if not args.no_large:
            meter_l = None if args.no_energy else EnergyMeter(torch)
            for dt_, runs, wu in (("f32", 2, 1), ("f64", 2, 0)):
                print(f"[bench] secondary n=65536 {dt_} path=True", file=sys.stderr, flush=True)
                sec_out[f"large_{dt_}_path_n65536"] = time_large(fw, torch, dt_, runs, wu, meter_l)
        print("[bench] secondary out of core n=32768", file=sys.stderr, flush=True)
        sec_out["ooc_f32_dist"] = time_ooc(fw, torch, runs=K)
        print("[bench] secondary out of core n=16384 with the path matrix", file=sys.stderr, flush=True)
        sec_out["ooc_f32_path"] = time_ooc(fw, torch, n=16384, S=4096, path=True, runs=K)
        print("[bench] secondary batched 10,000 graphs", file=sys.stderr, flush=True)
        sec_out["batched"] = time_batched(fw, torch, steps=K, warmup=Wu)
        print("[bench] secondary forward + backward", file=sys.stderr, flush=True)
        sec_out["fwd_bwd"] = time_fwd_bwd(fw, torch, steps=K, warmup=Wu)
        out["secondary"] = sec_out
    out["paper_context"] = {"note": "best measured GFLOPS over N in {4096..65536}, other hardware",
                            "f32": {"Xeon Phi KNL 7230": 1037, "Titan X (Pascal)": 972},
                            "f64": {"Xeon Phi KNL 7230": 501, "Titan X (Pascal)": 90}}
    if not args.no_cpu_baseline:
        t1 = single.join() if single is not None else None  # before the all-core runs
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.n)
        out["cpu_baseline"]["host"] = host_cpu()
        if not args.no_oracle_timings:
            print("[bench] oracle timings on the small workloads", file=sys.stderr, flush=True)
            out["cpu_baseline"]["oracle_timings"] = oracle_timings(fw, torch, sec_out, single_thread_s=t1,
                                                                   runs=args.sec_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
