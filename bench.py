"""Benchmark: SOR stress-majorization layout of a Barabasi-Albert graph,
n = 65,536, m = 3, 2-D, FP32, on one MI355X.

A step is one iteration of Algorithm 2 at omega = 1.5 with the safeguard on:
the Jacobi update and extrapolation, one pass over every vertex pair that takes
the next force at X~ and sums the safeguard f(X~) - f(X^H) (in 2-D once per
unordered pair, the library's default there), the select/termination kernel,
and the force pass at X^H when X~ was rejected (the first force, at X^0, is
inside the timed run).  The plan (distances and
weights) is built before the timed region, so inputs are resident in HBM.

value = n (n - 1) * steps / seconds   (pair interactions of the force pass)

Also reported: time-to-converge (res <= 1e-3) for omega = 1 and omega in
{1.5, 2, 2.5, 3} from the same start (speedup quoted at omega = 2.5, the
paper's w_p = 1.5), the same for the relaxation strategies of Sec. 5.2
(probabilistic, enumerating, per-vertex factors) and for the exact step H
(eq. 5 solved by conjugate gradients), the roofline of the fused force +
safeguard pass (HIP-event time) beside the plain force pass of omega = 1 runs
and the other kind of pass, and
the FP64 oracle's pair rate on a sample of rows on the host cores.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--dim 2] [--quick]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-interactions/s + time-to-converge (SOR-ω vs ω=1) at n=65,536, 1 MI355X"
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (packed-FMA issue)
PEAK_HBM_GBPS = 8000.0    # MI355X HBM3E
FLOPS_PER_PAIR = {2: 12, 3: 17}  # algorithmic flops of one ordered pair of the force pass
# algorithmic flops of the safeguard term of one unordered pair (the stress
# difference w (r~ - r^H)(r~ + r^H - 2d)), transcendentals (rsq, sqrt, rcp)
# counted as 0 flops as in the force term: 15 in 2-D, and 5 more in 3-D for the
# third coordinate of e, 2t - e and m (the pass over ordered pairs)
SG_FLOPS_PER_UNORDERED_PAIR = {2: 15, 3: 20}
# the pass over unordered pairs sums the bounds U = -2 sum_i e_i.F_i + sum c |e|^2
# and L = -2 sum_i e_i.F_i - sum w |e|^2 instead: per pair e = e_i - e_j (2),
# |e|^2 (3), and the two accumulating FMAs (4): 9 in 2-D, 12 in 3-D (the
# O(n) dot product e.F is left out)
SG_BOUNDS_FLOPS_PER_UNORDERED_PAIR = {2: 9, 3: 12}
# the library's default force pass for hop-count plans: once per unordered
# pair from a padded size of 24576 vertices (16384 in runs that extrapolate with
# the safeguard), else over every ordered pair (the faster one, 2-D and 3-D)
SYM_MIN_N_PAD = 24576
LW_SYM_MIN_N_PAD = 24576  # the exact step's L^W matvec over unordered pairs (2-D)
SYM_MIN_N_PAD_FUSED = 16384


def sym_default(dim, n, fused=True):
    return max(64, -(-n // 64) * 64) >= (SYM_MIN_N_PAD_FUSED if fused else SYM_MIN_N_PAD)
CSRC = os.path.join(ROOT, "paper_1711_01228_amd", "csrc")
# committed rocprofv3 traffic of the dominant kernel, with the source it was taken on
TRAFFIC = {True: (os.path.join(ROOT, "profiles", "force_safeguard_sym_ba65536_traffic.json"),
                  os.path.join(CSRC, "sl_sym.hip")),
           False: (os.path.join(ROOT, "profiles", "force_safeguard_ba65536_traffic.json"),
                   os.path.join(CSRC, "sl_kernels.hip"))}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(path):
    """Hash of a source's code with its comments and blank lines removed, so a
    counter record stays tied to the kernel it was taken on, not its prose."""
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = (" ".join(line.split()) for line in text.splitlines())
    return hashlib.sha256("\n".join(l for l in lines if l).encode()).hexdigest()[:16]


VALU = {True: (os.path.join(ROOT, "profiles", "force_safeguard_sym_ba65536_valu.json"),
                os.path.join(CSRC, "sl_sym.hip"))}


def measured_valu(dim, sym, n):
    """VALU utilisation of the fused pass from committed rocprofv3 counters
    (SQ_ACTIVE_INST_VALU over GRBM_GUI_ACTIVE), if they were taken on the
    current kernel source and this workload."""
    if sym not in VALU:
        return None
    path, src = VALU[sym]
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha") != kernel_hash(src) or rec.get("dim") != dim or rec.get("n", n) != n:
        return None
    return {k: rec[k] for k in ("valu_busy", "valu_issue_slots_per_unordered_pair", "counters") if k in rec}


def measured_traffic(dim, sym, n):
    """HBM bytes per launch of the fused pass from committed rocprofv3 counters,
    if they were taken on the current kernel source and this workload."""
    path, src = TRAFFIC[sym]
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha") != kernel_hash(src) or rec.get("dim") != dim or rec.get("n", n) != n:
        return None
    return rec.get("bytes_per_launch")


PROBE_KINDS = {"fma": 0, "rsq": 1, "sqrt": 2, "rcp": 3}


def probe_library():
    """libslprobe (include/slprobe.h), the calibration kernels of this benchmark."""
    import ctypes

    try:
        import torch  # noqa: F401  (one HIP runtime for torch and the library)
    except ImportError:
        pass
    from paper_1711_01228_amd import build_lib

    lib = ctypes.CDLL(build_lib.PROBE_LIB)
    d = ctypes.POINTER(ctypes.c_double)
    lib.slp_probe_rate.argtypes = [ctypes.c_int32, ctypes.c_void_p, d, d]
    lib.slp_probe_rate.restype = ctypes.c_int32
    return lib


def probe_rate(kind):
    """(lane operations per second, ms) of one instruction kind on the device."""
    import ctypes

    import torch

    per_s, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    st = probe_library().slp_probe_rate(PROBE_KINDS[kind], torch.cuda.current_stream().cuda_stream,
                                        ctypes.byref(per_s), ctypes.byref(ms))
    if st != 0:
        raise RuntimeError("slp_probe_rate(%s) failed with %d" % (kind, st))
    return per_s.value, ms.value


def measured_ceilings():
    """What this device sustains, beside its data-sheet peaks: plain FP32 FMAs
    (the build has no packed FP32) and the transcendentals of the force and
    safeguard terms, from the library's calibration kernels, and a 1 GiB
    device-to-device copy (read + write bytes over its HIP-event time)."""
    import torch

    res = {}
    fma, _ = probe_rate("fma")
    res["fp32_fma_TFLOPs"] = round(2.0 * fma / 1e12, 2)
    for k in ("rsq", "sqrt", "rcp"):
        res["%s_per_s" % k] = float("%.4g" % probe_rate(k)[0])
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        dst.copy_(src)
    b.record()
    b.synchronize()
    res["hbm_copy_GBps"] = round(5 * 2 * src.numel() * 4 / (a.elapsed_time(b) * 1e-3) / 1e9, 1)
    del src, dst
    return res


def host_cpu():
    """Model, logical CPUs and clock of the host, from lscpu (or /proc/cpuinfo)."""
    import subprocess

    info = {"model": "unknown", "cpus": os.cpu_count(), "mhz": None}
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True,
                             timeout=20).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            k, v = k.strip(), v.strip()
            if k == "Model name":
                info["model"] = v
            elif k == "CPU(s)":
                info["cpus"] = int(v)
            elif k in ("CPU max MHz", "CPU MHz") and info["mhz"] is None:
                info["mhz"] = float(v)
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    if info["mhz"] is None:  # the clock named in the model string (e.g. "@ 2.70GHz")
        import re

        m = re.search(r"@\s*([0-9.]+)\s*GHz", info["model"])
        if m:
            info["mhz"] = float(m.group(1)) * 1000.0
    if info["mhz"] is None:  # the current clock the kernel reports for the first CPU
        try:
            with open("/proc/cpuinfo") as f:
                for ln in f:
                    k, _, v = ln.partition(":")
                    if k.strip() == "cpu MHz":
                        info["mhz"] = float(v.strip())
                        info["mhz_source"] = "/proc/cpuinfo cpu MHz (current clock of CPU 0)"
                        break
        except (OSError, ValueError):
            pass
    return info


def oracle_threads():
    """Threads the oracle's OpenMP loops use in this process."""
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _oracle_rows_rate(g, X0, rows, block=512):
    """Pair rate of the oracle's Jacobi rows (eq. 5 row solves) for the given
    rows, their distance rows found block by block (never all at once)."""
    import numpy as np

    import oracle

    n = g.n
    dt = 0.0
    for a in range(0, len(rows), block):
        r = rows[a:a + block]
        Drows = oracle.sssp_rows(g.row_ptr, g.col_idx, r)
        t = time.perf_counter()
        oracle.h_jacobi_rows(Drows, r, X0)
        dt += time.perf_counter() - t
        del Drows
    return len(rows) * (n - 1) / dt, dt


def cpu_baseline(g, X0, target_s=12.0):
    """The FP64 oracle's Jacobi step on a sample of rows of the same graph, on
    all the threads this process gives it and (in a child process) on one."""
    import subprocess

    import numpy as np

    n = g.n
    rng = np.random.default_rng(0)
    rate0, _ = _oracle_rows_rate(g, X0, np.sort(rng.choice(n, 128, replace=False)))
    R = int(min(n, max(128, rate0 * target_s / (n - 1))))
    rows = np.sort(rng.choice(n, R, replace=False))
    rate, dt = _oracle_rows_rate(g, X0, rows)
    cores = oracle_threads()
    one = None
    code = ("import sys, numpy as np; sys.path.insert(0, %r); import bench; from paper_1711_01228_amd import inputs; "
            "g, X0 = inputs.ba65536(%d, n=%d); rows = np.sort(np.random.default_rng(1).choice(g.n, 64, replace=False)); "
            "print(bench._oracle_rows_rate(g, X0, rows)[0])" % (ROOT, X0.shape[1], n))
    try:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        out = subprocess.run([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                             env=env, text=True, timeout=300)
        one = float(out.stdout.strip().splitlines()[-1])
    except (OSError, ValueError, IndexError, subprocess.SubprocessError):
        pass
    return {"value": rate, "unit": "pair-interactions/s", "cores": cores, "kind": "oracle", "host": host_cpu(),
            "sample": "FP64 Jacobi step (eq. 5 row solves) for %d random rows x all %d columns of the same "
                      "BA graph and start, %.1f s on %d threads; distance rows (BFS) found in blocks of 512 rows "
                      "and not timed" % (R, n, dt, cores),
            "value_1_thread": one,
            "seconds_per_jacobi_step": float(n) * (n - 1) / rate}


def _oracle_runs_seconds(cases, threads=None):
    """Seconds of the oracle's Algorithm 2 run for each case (config, run, omega,
    tol, max_iter), in this process or, with `threads`, in a child process with
    OMP_NUM_THREADS = threads.  Returns [(seconds, iterations), ...]."""
    import subprocess

    if threads is not None:
        code = ("import sys, json; sys.path.insert(0, %r); import bench; "
                "print(json.dumps(bench._oracle_runs_seconds(%r)))" % (ROOT, cases))
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        out = subprocess.run([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                             env=env, text=True, timeout=3000)
        return json.loads(out.stdout.strip().splitlines()[-1])
    import oracle
    from paper_1711_01228_amd import inputs

    res = []
    for config, run, omega, tol, max_iter in cases:
        g, X0 = inputs.grid16(run) if config == 1 else inputs.er4096(run)
        D = oracle.apsp(g.row_ptr, g.col_idx)  # distances once per graph, not timed
        t = time.perf_counter()
        _, info = oracle.layout(D, X0, omega=omega, tol=tol, max_iter=max_iter)
        res.append((time.perf_counter() - t, info["iterations"]))
    return res


def bench_small_configs(seeds=20, full_oracle=False):
    """The grid (16 x 16, 200 iterations at omega 1 and 1.5) and Erdos-Renyi
    (n = 4096, mean degree 6, to res <= 1e-3 or 2,000 iterations over the omega
    sweep 1.0 .. 1.6) workloads over `seeds` seeds each (config c, run r: seed
    1000 c + r).  GPU: us per iteration (launch-bound sizes: device time of the
    run over its iterations) and time to tol (wall, plan excluded, one untimed
    run first); medians over the seeds.  Beside them the FP64 oracle runs the same
    layouts to the end on all threads of this process (the grid: every seed;
    Erdos-Renyi: seed 0 of every omega) and on one thread (the grid: every seed;
    Erdos-Renyi seed 0 at omega 1 only with full_oracle)."""
    import numpy as np
    import torch

    from paper_1711_01228_amd import binding, inputs

    out = {"seeds": seeds}
    # ---- grid 16 x 16, 200 iterations
    c1 = {}
    for om in (1.0, 1.5):
        us, wall, us_wg = [], [], []
        for r in range(seeds):
            g, X0 = inputs.grid16(r)
            Xd0 = torch.tensor(X0.astype(np.float32), device="cuda")
            with binding.Plan(g, 2) as plan:
                plan.run(Xd0.clone(), omega=om, tol=0.0, max_iter=200)
                X = Xd0.clone()
                torch.cuda.synchronize()
                t = time.perf_counter()
                info = plan.run(X, omega=om, tol=0.0, max_iter=200, final_stress=False)
                torch.cuda.synchronize()
                wall.append(time.perf_counter() - t)
                us.append(1e3 * info["run_ms"] / info["iterations"])
            # the same 200 iterations inside one workgroup (the batched layout of one graph)
            with binding.BatchPlan([g], 2) as bplan:
                bplan.run(Xd0.clone(), omega=om, tol=0.0, max_iter=200)
                tot, _ = bplan.run(Xd0.clone(), omega=om, tol=0.0, max_iter=200)
                us_wg.append(1e3 * tot["run_ms"] / max(tot["iterations"], 1))
        c1["omega=%g" % om] = {"us_per_iteration_median": round(float(np.median(us)), 2),
                               "us_per_iteration_range": [round(float(min(us)), 2), round(float(max(us)), 2)],
                               "seconds_200_iterations_median": round(float(np.median(wall)), 5),
                               "one_workgroup_us_per_iteration_median": round(float(np.median(us_wg)), 2)}
    out["grid16"] = c1
    # ---- Erdos-Renyi n = 4096 to tol
    c2 = {}
    omegas = (1.0, 1.2, 1.4, 1.6)
    per = {om: {"s": [], "it": [], "conv": 0} for om in omegas}
    for r in range(seeds):
        g, X0 = inputs.er4096(r)
        Xd0 = torch.tensor(X0.astype(np.float32), device="cuda")
        with binding.Plan(g, 2) as plan:
            for om in omegas:
                plan.run(Xd0.clone(), omega=om, tol=1e-3, max_iter=2000)
                X = Xd0.clone()
                torch.cuda.synchronize()
                t = time.perf_counter()
                info = plan.run(X, omega=om, tol=1e-3, max_iter=2000, final_stress=False)
                torch.cuda.synchronize()
                per[om]["s"].append(time.perf_counter() - t)
                per[om]["it"].append(info["iterations"])
                per[om]["conv"] += int(info["converged"])
    base = np.array(per[1.0]["s"])
    for om in omegas:
        sec, it = np.array(per[om]["s"]), np.array(per[om]["it"])
        c2["omega=%g" % om] = {"seconds_to_tol_median": round(float(np.median(sec)), 5),
                               "iterations_median": float(np.median(it)),
                               "us_per_iteration_median": round(float(np.median(1e6 * sec / it)), 2),
                               "converged": "%d/%d" % (per[om]["conv"], seeds),
                               "speedup_vs_omega1_median": round(float(np.median(base / sec)), 3)}
    out["er4096"] = c2
    # ---- the oracle beside it
    cases1 = [(1, r, om, 0.0, 200) for om in (1.0, 1.5) for r in range(seeds)]
    cases2 = [(2, 0, om, 1e-3, 2000) for om in omegas]
    orc = {"threads": oracle_threads(), "host": host_cpu()}
    t1 = _oracle_runs_seconds(cases1)
    orc["grid16_seconds_median"] = {"omega=%g" % om: round(float(np.median([t for (c, r, o, _, _), (t, _) in
                                                                           zip(cases1, t1) if o == om])), 5)
                                    for om in (1.0, 1.5)}
    t1s = _oracle_runs_seconds(cases1, threads=1)
    orc["grid16_seconds_median_1_thread"] = {"omega=%g" % om: round(float(np.median(
        [t for (c, r, o, _, _), (t, _) in zip(cases1, t1s) if o == om])), 5) for om in (1.0, 1.5)}
    t2 = _oracle_runs_seconds(cases2)
    orc["er4096_seed0"] = {"omega=%g" % om: {"seconds_to_tol": round(t, 3), "iterations": it}
                           for om, (t, it) in zip(omegas, t2)}
    if full_oracle:
        (t, it), = _oracle_runs_seconds([(2, 0, 1.0, 1e-3, 2000)], threads=1)
        orc["er4096_seed0_1_thread"] = {"omega=1": {"seconds_to_tol": round(t, 3), "iterations": it}}
    out["oracle"] = orc
    return out


def bench_batch(omega, count=2048):
    """2,048 graphs (n ~ U[16, 1024]: grids, random trees, Erdos-Renyi giant
    components of mean degree 4), omega = 1.5 with the safeguard, each graph to
    res <= 1e-3, in one persistent captured launch with autotuned tile shapes."""
    import numpy as np
    import torch

    from paper_1711_01228_amd import binding, inputs

    gs, xs = inputs.batch_of_graphs(count)
    X0 = torch.tensor(np.concatenate(xs).astype(np.float32), device="cuda")
    t = time.perf_counter()
    plan = binding.BatchPlan(gs, 2)
    plan_s = time.perf_counter() - t
    t = time.perf_counter()
    cfg = plan.tune(X0, omega=omega, tol=1e-3, max_iter=3000)  # the workgroup size on whole runs to tol
    tune_s = time.perf_counter() - t
    X = X0.clone()
    plan.run(X, omega=omega, tol=1e-3, max_iter=3000)  # warm (graph capture)
    X = X0.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    tot, per = plan.run(X, omega=omega, tol=1e-3, max_iter=3000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    plan.close()
    its = np.array([p["iterations"] for p in per])
    ns = np.array([g.n for g in gs], dtype=np.float64)
    pairs = float(np.sum(ns * (ns - 1) * its))
    return {"graphs": count, "vertices": int(ns.sum()), "pairs_per_pass": float(np.sum(ns * (ns - 1))),
            "seconds": round(wall, 4), "device_ms": round(tot["run_ms"], 3), "plan_s": round(plan_s, 3),
            "plan_device_ms": round(tot["plan_ms"], 3),
            "tune_s": round(tune_s, 3),
            "pair_interactions_per_s": pairs / wall, "iterations_mean": float(its.mean()),
            "iterations_max": int(its.max()), "all_converged": bool(tot["converged"]),
            "rejected_total": int(tot["rejected"]), "tuned_config": cfg.tolist()}


# The paper writes the extrapolation as X~ = (1 + w_p) X^H - w_p X^k, so its
# factor w_p is omega - 1 here; its headline setting w_p = 1.5 is omega = 2.5.
SOR_OMEGAS = (1.5, 2.0, 2.5, 3.0)
PAPER_OMEGA = 2.5


def time_to_converge(plan, Xdev0, omegas=(1.0,) + SOR_OMEGAS):
    """Wall time to res <= 1e-3 from the same start for each fixed omega (one
    untimed run first, so that every timed run replays captured graphs), and
    the speedup of omega = 2.5 and of the fastest omega over omega = 1."""
    import numpy as np
    import torch

    ttc = {}
    for om in omegas:
        # untimed run with a trace: how each safeguard decision was taken
        warm = plan.run(Xdev0.clone(), omega=om, tol=1e-3, max_iter=3000, trace=True)
        tr = warm["trace"][:warm["iterations"]]
        decided = tr[:, 1] >= 0
        by_bounds = int(np.sum(decided & np.isnan(tr[:, 2])))
        exact_after_bounds = int(np.sum(decided & ~np.isnan(tr[:, 2]) & ~np.isnan(tr[:, 5])))
        X = Xdev0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = plan.run(X, omega=om, tol=1e-3, max_iter=3000, final_stress=False)
        torch.cuda.synchronize()
        w = time.perf_counter() - t
        ttc["omega=%g" % om] = {"seconds": round(w, 4), "device_s": round(r["run_ms"] / 1e3, 4),
                                "iterations": r["iterations"], "converged": bool(r["converged"]),
                                "rejected": r["rejected"], "final_residual": r["residual"],
                                "final_stress": plan.stress(X)}
        if om != 1.0:
            ttc["omega=%g" % om]["safeguard_decisions"] = {"by_bounds": by_bounds,
                                                           "exact_pass": exact_after_bounds,
                                                           "total": int(np.sum(decided))}
        log("time-to-converge omega=%g: %s" % (om, ttc["omega=%g" % om]))
    base = ttc["omega=1"]["seconds"]
    best = min((o for o in omegas if o != 1.0), key=lambda o: ttc["omega=%g" % o]["seconds"])
    ttc["speedup"] = round(base / ttc["omega=%g" % PAPER_OMEGA]["seconds"], 3)
    ttc["speedup_omega"] = PAPER_OMEGA
    ttc["best_omega"] = best
    ttc["speedup_best"] = round(base / ttc["omega=%g" % best]["seconds"], 3)
    ttc["tol"] = 1e-3
    return ttc


def bench_strategies(plan, Xdev0, n):
    """The relaxation strategies of Sec. 5.2 on the same plan and start: per
    iteration device time (20 iterations, tol 0) and time to res <= 1e-3."""
    import numpy as np
    import torch

    from paper_1711_01228_amd import binding

    rng = np.random.default_rng(77)
    cases = {
        "fixed omega=1.5": dict(omega=1.5),
        "fixed omega=2.5": dict(omega=2.5),
        "probabilistic (seed 5)": dict(strategy="auto", seed=5),
        "enumerating": dict(strategy="enum"),
        "per-vertex omega_i ~ U[1,2] (seed 77)": dict(
            omega_vertex=torch.tensor(rng.uniform(1.0, 2.0, n).astype(np.float32), device="cuda")),
    }
    res = {}
    for name, kw in cases.items():
        X = Xdev0.clone()
        r = plan.run(X, tol=0.0, max_iter=20, **kw)
        per_it = r["run_ms"] / r["iterations"]
        X = Xdev0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = plan.run(X, tol=1e-3, max_iter=3000, final_stress=False, **kw)
        torch.cuda.synchronize()
        w = time.perf_counter() - t
        res[name] = {"ms_per_iteration": round(per_it, 4), "seconds_to_tol": round(w, 4),
                     "iterations": r["iterations"], "converged": bool(r["converged"]), "rejected": r["rejected"],
                     "final_residual": r["residual"], "final_stress": plan.stress(X)}
        log("strategy %s: %s" % (name, res[name]))
    return res


def bench_exact(plan, Xdev0, n, ms, dim=2):
    """The paper's exact step H (eq. 5 solved by preconditioned CG on the
    device) on the same plan and start: time to res <= 1e-3 at omega = 1,
    1.5 and 2.5, and the HBM roofline of the L^W matvec (one distance byte per
    unordered pair for the library's default pass at this size, else per ordered
    pair)."""
    import torch

    res = {}
    for om in (1.0, 1.5, PAPER_OMEGA):
        X = Xdev0.clone()
        plan.run(X, omega=om, tol=0.0, max_iter=1, ordering="exact")  # warm (allocation, capture)
        X = Xdev0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = plan.run(X, omega=om, tol=1e-3, max_iter=500, ordering="exact", final_stress=False)
        torch.cuda.synchronize()
        w = time.perf_counter() - t
        res["omega=%g" % om] = {"seconds_to_tol": round(w, 4), "iterations": r["iterations"],
                                "cg_steps": r["inner_iterations"], "converged": bool(r["converged"]),
                                "rejected": r["rejected"], "final_residual": r["residual"],
                                "final_stress": plan.stress(X)}
        log("exact omega=%g: %s" % (om, res["omega=%g" % om]))
    res["speedup"] = round(res["omega=1"]["seconds_to_tol"] / res["omega=%g" % PAPER_OMEGA]["seconds_to_tol"], 3)
    res["speedup_omega"] = PAPER_OMEGA
    t_lw = ms["lw_matvec"] * 1e-3
    # the library's default matvec: over unordered pairs in 2-D from n_pad 24576
    # (one distance byte per unordered pair), else over every ordered pair
    lw_sym = dim == 2 and max(64, -(-n // 64) * 64) >= LW_SYM_MIN_N_PAD
    lw_bytes = float(n) * (n - 1) / 2 if lw_sym else float(n) * n
    gbs = lw_bytes / t_lw / 1e9
    res["lw_matvec_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                                 "frac": round(gbs / PEAK_HBM_GBPS, 4),
                                 "kernel": "k_lw_sym + k_lw_sym_reduce (unordered pairs)" if lw_sym else "k_lw",
                                 "kernel_ms": round(ms["lw_matvec"], 4), "algorithmic_bytes_per_launch": lw_bytes}
    res["inner_tol"] = 1e-6
    return res


def bench_diff(steps=3):
    """Differentiation: ER n=16,384, mean degree 8, edge lengths 1 +- 0.1, 100
    unrolled iterations at omega = 1.5 with checkpoints every 10; loss = stress
    against hop distances.  Forward = shortest paths for the current lengths +
    unrolled iterations; backward = gradients w.r.t. X0 and every edge length."""
    import numpy as np
    import torch

    from paper_1711_01228_amd import autograd as ag
    from paper_1711_01228_amd import inputs

    n, K = 16384, 100
    g = inputs.erdos_renyi(n, n * 8 // 2, inputs.workload_seed(5))
    rng = np.random.default_rng(inputs.workload_seed(5) + 1)
    ln = (1.0 + rng.uniform(-0.1, 0.1, g.num_edges)).astype(np.float32)
    X0 = inputs.uniform_positions(n, 2, inputs.workload_seed(5) + 2, 0.0, float(np.sqrt(n)))
    t = time.perf_counter()
    lay = ag.DifferentiableLayout(g, 2, ln)
    plan_s = time.perf_counter() - t
    fw, bw, tot = [], [], []
    for rep in range(steps + 1):
        X0t = torch.tensor(X0.astype(np.float32), device="cuda", requires_grad=True)
        lt = torch.tensor(ln, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X = ag.unrolled_layout(X0t, lt, lay, omega=1.5, iters=K, ckpt_every=10)
        loss = ag.stress_loss(X, lay)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep > 0:  # the first pass allocates the tape and adjoint buffers
            fw.append(t1 - t0)
            bw.append(t2 - t1)
            tot.append(t2 - t0)
    gX0 = X0t.grad.cpu().numpy().astype(np.float64)
    glen = lt.grad.cpu().numpy().astype(np.float64)
    lay.close()
    pairs = float(n) * (n - 1)
    return {"workload": "Erdos-Renyi n=%d, %d edges (mean degree 8), lengths U[0.9,1.1], start U[0,%d]^2, "
                        "%d unrolled iterations at omega=1.5 with safeguard, checkpoints every 10, stress loss vs "
                        "hop distances; gradients w.r.t. X0 and every edge length" % (n, g.num_edges, int(np.sqrt(n)), K),
            "plan_s": round(plan_s, 3), "forward_s": round(float(np.median(fw)), 4),
            "backward_s": round(float(np.median(bw)), 4), "step_s": round(float(np.median(tot)), 4),
            "steps_timed": steps, "loss": float(loss.detach()),
            "forward_pair_interactions_per_s": K * pairs / float(np.median(fw)),
            "grad_translation_residual": float(np.abs(gX0.sum(0)).max() / np.abs(gX0).sum()),
            "grad_len_norm": float(np.linalg.norm(glen)), "grad_x0_norm": float(np.linalg.norm(gX0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3))
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--omega", type=float, default=1.5)
    ap.add_argument("--quick", action="store_true", help="skip time-to-converge and the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D run of the same workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched small-graph run")
    ap.add_argument("--no-strategies", action="store_true", help="skip the relaxation-strategy comparison")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact-step (eq. 5 solved) comparison")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation workload")
    ap.add_argument("--no-small", action="store_true", help="skip the grid / Erdos-Renyi workloads over 20 seeds")
    ap.add_argument("--full-oracle", action="store_true",
                    help="also run the oracle on one thread to convergence on the Erdos-Renyi workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1711_01228_amd import binding, build_lib, inputs

    assert os.path.exists(build_lib.LIB), "libsorlayout.so is not built"
    torch.cuda.set_device(0)
    n, dim = args.n, args.dim
    t0 = time.perf_counter()
    g, X0 = inputs.ba65536(dim=dim, n=n)
    log("graph: BA n=%d m=3, %d edges, max degree %d (%.1f s)" % (g.n, g.num_edges, np.diff(g.row_ptr).max(),
                                                               time.perf_counter() - t0))
    Xdev0 = torch.tensor(X0.astype(np.float32), device="cuda")
    # the process's first plan also loads the library's code objects: it is
    # reported beside a second plan of the same graph, made in the warm process
    plan = binding.Plan(g, dim)
    plan_ms_first = plan.run(Xdev0.clone(), omega=1.0, tol=0.0, max_iter=0)["plan_ms"]
    plan.close()
    plan = binding.Plan(g, dim)
    X = Xdev0.clone()
    info = plan.run(X, omega=args.omega, tol=0.0, max_iter=max(args.warmup, 1))  # warmup (+ graph capture)
    plan_ms = info["plan_ms"]
    log("plan %.1f ms (first plan of the process %.1f ms); warmup %d steps %.1f ms"
        % (plan_ms, plan_ms_first, info["iterations"], info["run_ms"]))

    # ---- timed region: K steps
    X = Xdev0.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    # the stress of the result is a report, not a step: it is evaluated after the timed region
    info = plan.run(X, omega=args.omega, tol=0.0, max_iter=args.steps, final_stress=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    assert info["iterations"] == args.steps, info
    pairs = float(n) * (n - 1)
    value = pairs * args.steps / wall
    log("timed: %d steps %.3f s wall (%.3f s device), %.4g pair-interactions/s" % (args.steps, wall,
                                                                                   info["run_ms"] / 1e3, value))

    # ---- roofline of the dominant kernel: the fused force + safeguard pass of
    # the default kind (HIP events on the kernels' stream); the force pass of
    # omega = 1 iterations and the other kind beside it
    ms = plan.profile(Xdev0, omega=args.omega, reps=5)
    sym = sym_default(dim, n)
    t_fs = (ms["force_safeguard_sym"] if sym else ms["force_safeguard"]) * 1e-3
    sg_flops = (SG_BOUNDS_FLOPS_PER_UNORDERED_PAIR if sym else SG_FLOPS_PER_UNORDERED_PAIR)[dim]
    flops = FLOPS_PER_PAIR[dim] * pairs + sg_flops * pairs / 2
    achieved = flops / t_fs / 1e12
    t_force = (ms["force_sym"] if sym else ms["force"]) * 1e-3
    a_force = FLOPS_PER_PAIR[dim] * pairs / t_force / 1e12
    abytes = float(n) * (n - 1) / 2 if sym else float(n) * n  # d read once per unordered / ordered pair
    other = {"kernel": "k_force_sg (fused) and k_force over every ordered pair" if sym else
             "k_force_sym<2, 1> / <2, 0> + k_sym_reduce over unordered pairs",
             "fused_ms": round(ms["force_safeguard"] if sym else ms["force_safeguard_sym"], 4),
             "force_ms": round(ms["force"] if sym else ms["force_sym"], 4)}
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": measured_traffic(dim, sym, n),
                "kernel": ("k_force_sym<2, 1> + k_sym_reduce<2> (unordered pairs, bounds of the safeguard)" if sym
                           else "k_force_sg (ordered pairs)"),
                "kernel_ms": round(t_fs * 1e3, 4),
                "flops_per_launch": flops,
                "flops_per_unit": {"ordered_pair_force": FLOPS_PER_PAIR[dim],
                                   "unordered_pair_safeguard": sg_flops},
                "safeguard": ("bounds U >= f(X~) - f(X^H) >= L; the exact difference only when they leave "
                              "its sign open" if sym else "the exact difference, pair by pair"),
                "algorithmic_bytes_per_launch": abytes,
                "hbm_GBps_algorithmic": round(abytes / t_fs / 1e9, 1),
                "force_pass": {"kernel": ("k_force_sym<2, 0> + k_sym_reduce<2>" if sym else "k_force") +
                               " (omega = 1 iterations; after a rejection)",
                               "kernel_ms": round(t_force * 1e3, 4), "TFLOPs": round(a_force, 3),
                               "frac": round(a_force / PEAK_FP32_TFLOPS, 4)},
                "other_kind": other,
                "separate_passes_ms": round(ms["force"] + ms["safeguard"], 4),
                "exact_variant_ms": round(ms["force_safeguard_sym_exact"], 4) if sym else None,
                "step_kernel_ms": {k: round(v, 4) for k, v in ms.items()},
                "measured_ceilings": measured_ceilings()}
    roofline["frac_of_measured_fma"] = round(achieved / roofline["measured_ceilings"]["fp32_fma_TFLOPs"], 4)
    roofline["valu"] = measured_valu(dim, sym, n)
    if roofline["traffic"]:
        roofline["traffic_over_algorithmic"] = round(roofline["traffic"] / abytes, 3)
    log("kernels (ms):", ms)
    log("measured ceilings:", roofline["measured_ceilings"])

    out = {"metric": METRIC, "value": value, "unit": "pair-interactions/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "Barabasi-Albert n=%d m=3 (%d edges), %d-D, start U[0,1]^%d, omega=%.2f "
                                  "with safeguard, Jacobi ordering" % (n, g.num_edges, dim, dim, args.omega),
                      "n": n, "dim": dim, "omega": args.omega, "step": "one iteration of Algorithm 2"},
           "plan_ms": plan_ms, "plan_ms_first_in_process": round(plan_ms_first, 3),
           # the all-pairs BFS (row A0) writes one distance byte per pair; W follows from it
           "plan_apsp": {"kernels": "k_bfs_pairs, k_bfs_gather/store (8,192 sources per sweep; W summed in the store) + k_weights_from_partials",
                         "bytes_written": float(n) * n, "GBps": round(float(n) * n / (plan_ms * 1e-3) / 1e9, 1),
                         "frac_of_hbm_peak": round(float(n) * n / (plan_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4)},
           "roofline": roofline}

    # ---- time to converge: SOR-omega vs omega = 1 at equal final residual
    if not args.quick:
        out["time_to_converge"] = time_to_converge(plan, Xdev0)
        if not args.no_strategies:
            out["strategies"] = bench_strategies(plan, Xdev0, n)
        if not args.no_exact:
            out["exact"] = bench_exact(plan, Xdev0, n, ms, dim)
    plan.close()
    del plan

    # ---- the same workload in 3-D (float4 iterates)
    if not args.quick and not args.no_3d and dim == 2:
        g3, X03 = inputs.ba65536(dim=3, n=n)
        X3dev0 = torch.tensor(X03.astype(np.float32), device="cuda")
        plan3 = binding.Plan(g3, 3)
        X = X3dev0.clone()
        plan3.run(X, omega=args.omega, tol=0.0, max_iter=max(args.warmup, 1))
        X = X3dev0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = plan3.run(X, omega=args.omega, tol=0.0, max_iter=args.steps, final_stress=False)
        torch.cuda.synchronize()
        w3 = time.perf_counter() - t
        ms3 = plan3.profile(X3dev0, omega=args.omega, reps=5)
        ttc3 = time_to_converge(plan3, X3dev0)
        plan3.close()
        sym3 = sym_default(3, n)
        t3 = ms3["force_safeguard_sym"] if sym3 else ms3["force_safeguard"]
        sg3 = (SG_BOUNDS_FLOPS_PER_UNORDERED_PAIR if sym3 else SG_FLOPS_PER_UNORDERED_PAIR)[3]
        a3 = (FLOPS_PER_PAIR[3] * pairs + sg3 * pairs / 2) / (t3 * 1e-3) / 1e12
        out["dim3"] = {"value": pairs * args.steps / w3, "ms_per_step": w3 * 1e3 / args.steps,
                       "fused_kernel": ("k_force_sym<3, 1> + k_sym_reduce<3> (unordered pairs, bounds)" if sym3
                                        else "k_force_sg<3> (ordered pairs)"),
                       "fused_kernel_ms": round(t3, 4), "fused_TFLOPs": round(a3, 3),
                       "fused_frac": round(a3 / PEAK_FP32_TFLOPS, 4),
                       "step_kernel_ms": {k: round(v, 4) for k, v in ms3.items()}, "time_to_converge": ttc3}
        log("3-D:", out["dim3"])
    # ---- differentiation: gradients through 100 unrolled iterations at n = 16,384
    if not args.quick and not args.no_diff:
        out["differentiation"] = bench_diff()
        log("differentiation:", out["differentiation"])
    # ---- the small workloads over 20 seeds, the oracle beside them
    if not args.quick and not args.no_small:
        out["small_configs"] = bench_small_configs(full_oracle=args.full_oracle)
        log("small configs:", out["small_configs"])
    # ---- batched: 2,048 small graphs, one persistent launch, each to its own tol
    if not args.quick and not args.no_batch:
        out["batched"] = bench_batch(args.omega)
        log("batched:", out["batched"])
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = src.numel() * 4
        del src, dst

    if not args.quick and not args.no_cpu:
        cb = cpu_baseline(g, X0)
        if "time_to_converge" in out:  # omega = 1 takes one Jacobi step per iteration and no safeguard
            it1 = out["time_to_converge"]["omega=1"]["iterations"]
            cb["time_to_converge_omega1_extrapolated_s"] = round(cb["seconds_per_jacobi_step"] * it1, 2)
            cb["extrapolation"] = ("the oracle's s per Jacobi step x the GPU's %d iterations to res <= 1e-3 at "
                                   "omega = 1 (extrapolated, not run)" % it1)
        out["cpu_baseline"] = cb
        log("cpu baseline:", cb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
