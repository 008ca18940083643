"""Benchmark: noiseless LR-QAOA state-vector simulation on one MI355X.

Workload: K_32 weighted complete graph (seed 2, weights uniform on
{0.1..1.0}), p = 3, midpoint linear ramp with D_gamma = D_beta = 0.6,
complex64 state (32 GiB) + int32 cost diagonal (16 GiB).  One step runs the
whole hot path: cost diagonal, forward circuit with fused <C>/norm readout,
10,000 shots, and the forward+adjoint gradient.  The headline value is
amplitude-layer updates per second of the forward circuit, 2^n p / t_fwd,
measured inside every timed step with HIP events on the library's stream.

Also reported: the same forward and gradient in complex128 (and the
complex64 errors against it), the forward+adjoint / forward time ratio, the
algorithmic HBM bandwidth of the dominant kernel against the 8 TB/s peak,
the device's own streaming ceilings (the library's probe kernels), and the
CPU oracle timed on the host (a bounded sample, see cpu_baseline).  Side
runs in the same line (not part of the headline value): the store mode of
the adjoint (per-pass checkpoints, 160 GiB at n = 32), the exact cut-value
histogram of the final state, the complement-symmetric half-state layout,
the 512-circuit batched forward+adjoint in both precisions, the largest
sizes (K_34 forward with 100,000 shots; K_33 forward+adjoint), the
depolarizing-noise trajectories (K_12, p = 10) and the 30-qubit depth sweep
(K_30, seed 5, p = 3, 6, 10, 50, 100).

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-c128] [--no-sym]
                       [--no-store] [--no-batch] [--no-huge] [--no-noise] [--no-sweep30] [--no-window]
                       [--noise-only] [--window-only]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak: 256 CUs x 4 SIMDs x 32 lanes x 2 flops (FMA) x 2.4 GHz.  The
# build emits no packed FP32 instructions, but the unpacked FMAs reach this
# rate (the mixer-window probe's butterflies run at ~97 TFLOP/s, above the
# 78.6 that one FMA per 16 lanes per clock would allow).
FP32_VECTOR_TFLOPS = 157.3
KERNEL_SOURCES = ["paper_2604_26423_amd/csrc/pass.hip", "paper_2604_26423_amd/csrc/tiles.h",
                  "paper_2604_26423_amd/csrc/device.h",
                  "paper_2604_26423_amd/csrc/internal.h", "paper_2604_26423_amd/csrc/plan.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter runs, or None
    when the file is absent or the kernel sources changed since it was written."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def device_ceiling(torch, Q, gib: int = 4):
    """Streaming rates of the library's probe kernels (include/qs_probe.h) over
    `gib` GiB buffers: read, write, copy and in-place update, each the best of
    plain and nontemporal accesses and of 1 or 4 16-byte elements per thread."""
    nb = gib << 30
    a = torch.zeros(nb // 8, dtype=torch.complex64, device="cuda")
    b = torch.ones(nb // 8, dtype=torch.complex64, device="cuda")
    st = torch.cuda.current_stream()
    out = {}
    nt = Q.QS_PROBE_NT_LOAD | Q.QS_PROBE_NT_STORE
    for kind in ("read", "write", "copy", "update"):
        best = None
        for flags in (0, nt):
            for unroll in (1, 4):
                ms, by = Q.qs_bandwidth_probe(Q.PROBE_KINDS[kind], a, b, nb, reps=5, flags=flags, unroll=unroll,
                                              stream=st)
                gbs = by / (ms * 1e-3) / 1e9
                if best is None or gbs > best["gbs"]:
                    best = {"gbs": round(gbs, 1), "ms": round(ms, 4), "bytes": by,
                            "nontemporal": flags != 0, "elems_per_thread": unroll}
        out[kind] = best
    del a, b
    torch.cuda.empty_cache()
    out["copy_ceiling_gbs"] = max(out["copy"]["gbs"], out["update"]["gbs"])
    return out


def window_microbench(torch, Q, n: int = 30):
    """One four-qubit mixer window applied to two complex64 vectors of 2^n
    amplitudes (the two vectors of a reverse pass), `windows` times per load:
    tangent-form butterflies on the vector ALUs against the same product as a
    real 16 x 16 matrix on the FP32 matrix cores (include/qs_probe.h).
    windows = 8 is about the arithmetic per byte of a reverse junction."""
    a = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    rows = []
    for windows in (1, 8, 32):
        row = {"windows": windows}
        for kind in ("window_valu", "window_mfma"):
            a.normal_(0.0, 0.01)
            b.normal_(0.0, 0.01)
            ms, by = Q.qs_bandwidth_probe(Q.PROBE_KINDS[kind], a, b, 8 << n, reps=3, n=n, windows=windows,
                                          stream=st)
            # butterfly FLOPs of the product: 4 qubits x 2 FMAs per amplitude per window, two vectors
            flops = 2.0 ** n * 2 * windows * 4 * 4
            row[kind] = {"ms": round(ms, 4), "gbs": round(by / (ms * 1e-3) / 1e9, 1),
                         "butterfly_tflops": round(flops / (ms * 1e-3) / 1e12, 2)}
        row["mfma_over_valu_time"] = round(row["window_mfma"]["ms"] / row["window_valu"]["ms"], 3)
        log(f"window probe, {windows} per load: butterflies {row['window_valu']['ms']:.2f} ms, "
            f"matrix cores {row['window_mfma']['ms']:.2f} ms")
        rows.append(row)
    del a, b
    torch.cuda.empty_cache()
    return {"n": n, "vectors": 2, "qubits_per_window": 4, "rows": rows}


def host_info() -> dict:
    """CPU model, logical CPUs and available memory of the host."""
    info = {"cpu_model": None, "host_logical_cpus": os.cpu_count(), "host_mem_available_gib": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable:"):
                    info["host_mem_available_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


def single_thread_oracle(n: int, seed: int, tzz, tx) -> float:
    """Seconds of the oracle's forward at n qubits on one thread, in a child
    process started with OMP_NUM_THREADS=1 (no GPU use in the child)."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r); import oracle, workloads; "
            "w = workloads.complete_graph_tenths(%d, %d); t = time.perf_counter(); "
            "oracle.simulate(%d, w, %r, %r, mode=0); print(time.perf_counter() - t)"
            % (ROOT, n, seed, n, [float(x) for x in tzz], [float(x) for x in tx]))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    return float(r.stdout.strip().splitlines()[-1])


def symmetric_run(torch, Simulator, w, tzz, tx, exp_c_full, stream):
    """The same workload in the complement-symmetric layout (half state)."""
    sim = Simulator(w, "c64", symmetric=True)
    n = sim.n
    p = len(tzz)
    tf, ta = [], []
    for _ in range(4):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        e, _ = sim.forward(tzz, tx)
        e1.record(stream)
        sim.adjoint(tzz, tx)
        e2.record(stream)
        torch.cuda.synchronize()
        tf.append(e0.elapsed_time(e1))
        ta.append(e1.elapsed_time(e2))
    t_fwd, t_adj = float(sorted(tf[1:])[1]), float(sorted(ta[1:])[1])
    log(f"symmetric layout: forward {t_fwd:.1f} ms, forward+adjoint {t_adj:.1f} ms")
    # algorithmic bytes of the half state: read C and psi, write psi per layer (layer 1 skips the read)
    alg = 2.0 ** (n - 1) * (p * 20 - 8)
    out = {"forward_ms": round(t_fwd, 3), "forward_plus_adjoint_ms": round(t_adj, 3),
           "amp_layer_per_s": 2.0 ** n * p / (t_fwd * 1e-3),
           "forward_useful_hbm_frac": round(alg / (t_fwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "state_gib": 2.0 ** (n - 1) * 8 / 2 ** 30,
           "exp_c_rel_diff_vs_full_layout": abs(e - exp_c_full) / exp_c_full}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def batch_run(torch, workloads, stream, cpu: bool):
    """512 uneven circuits (n = 14..22, p in {3, 5, 10}): forward + adjoint
    gradient of all of them in one persistent launch, in complex64 (timed) and
    in complex128 (the per-circuit reference for the complex64 errors)."""
    import numpy as np
    from paper_2604_26423_amd import Batch
    items = workloads.batch()
    inst = [(it.weights(), it.p) for it in items]
    ang = []
    for it in items:
        g = [(k - 0.5) / it.p * it.delta_gamma for k in range(1, it.p + 1)]
        b = [(1 - (k - 0.5) / it.p) * it.delta_beta for k in range(1, it.p + 1)]
        ang.append((2.0 * np.asarray(g), -2.0 * np.asarray(b)))
    tzz, tx = [a[0] for a in ang], [a[1] for a in ang]
    res = {}
    for prec in ("c64", "c128"):
        bt = Batch(inst, prec)
        ts = []
        for _ in range(4):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            e, gzz, gx = bt.forward_grad(tzz, tx)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        res[prec] = (float(np.median(ts[1:])), e, gzz, gx, list(bt.cmax))
        bt.close()
        del bt
        torch.cuda.empty_cache()
    t, e, gzz, gx, cmax = res["c64"]
    t128, e128, gzz128, gx128, _ = res["c128"]
    amp_layers = sum(float(1 << it.n) * it.p for it in items)
    # per-circuit complex64 errors against the complex128 batch: <C> relative,
    # gradient relative to the circuit's largest gradient component
    e_err = np.abs(np.asarray(e) - np.asarray(e128)) / np.abs(np.asarray(e128))
    g_err = np.array([max(np.abs(a - c).max(), np.abs(b - d).max()) / max(np.abs(c).max(), np.abs(d).max())
                      for a, b, c, d in zip(gzz, gx, gzz128, gx128)])
    log(f"batch: {len(items)} circuits, {amp_layers / 1e9:.2f}e9 amp-layers, forward+adjoint {t:.2f} ms "
        f"(complex128 {t128:.2f} ms); complex64 <C> error max {e_err.max():.2e}, gradient max {g_err.max():.2e}")
    out = {"circuits": len(items), "forward_plus_adjoint_ms": round(t, 3), "circuits_per_s": len(items) / (t * 1e-3),
           "amp_layer_per_s_fwd_adj": amp_layers / (t * 1e-3),
           "mean_r_exact": float(np.mean([ei / (cm / 10) for ei, cm in zip(e, cmax)])),
           "c128_forward_plus_adjoint_ms": round(t128, 3),
           "c64_vs_c128": {"exp_c_rel_err_max": float(e_err.max()), "exp_c_rel_err_median": float(np.median(e_err)),
                           "grad_rel_err_max": float(g_err.max()), "grad_rel_err_median": float(np.median(g_err))}}
    if cpu:
        import oracle
        k = 3
        t0 = time.perf_counter()
        for it, (a, c) in zip(items[:k], ang[:k]):
            oracle.adjoint(it.n, it.weights(), a, c)
        tc = time.perf_counter() - t0
        out["cpu_oracle"] = {"circuits_per_s": k / tc, "cores": oracle.num_threads(), "kind": "oracle",
                             "sample": f"the first {k} circuits of the batch (n = "
                                       f"{', '.join(str(it.n) for it in items[:k])}), gate-by-gate adjoint, "
                                       f"complex128, {tc:.1f} s"}
    return out


def mem_used(torch) -> int:
    free, total = torch.cuda.mem_get_info()
    return total - free


def huge_run(torch, workloads, Simulator, linear_ramp, to_gate_angles, stream):
    """The largest sizes: K_34 (complex64, 128 GiB state + 64 GiB diagonal)
    forward with 100,000 shots, and K_33 forward+adjoint in uncompute mode
    (two 64 GiB state vectors + 32 GiB diagonal)."""
    import numpy as np
    out = {}
    for run, grad in ((workloads.HUGE, False), (workloads.HUGE_GRAD, True)):
        n, p = run.n, run.p
        g, b = linear_ramp(p, run.delta_gamma, run.delta_beta, "midpoint")
        tzz, tx = to_gate_angles(g, b, "paper")
        base = mem_used(torch)
        sim = Simulator(run.weights(), "c64")
        if grad:
            sim.lam = torch.empty_like(sim.psi)
        tf, ta, tsm = [], [], []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            e, _ = sim.forward(tzz, tx)
            e1.record(stream)
            if grad:
                sim.adjoint(tzz, tx)
            else:
                shots = sim.sample(run.shots, run.seed, on_device=True)
            e2.record(stream)
            torch.cuda.synchronize()
            tf.append(e0.elapsed_time(e1))
            (ta if grad else tsm).append(e1.elapsed_time(e2))
        peak = mem_used(torch) - base
        t_fwd = float(np.median(tf))
        alg = 20.0 * p * 2.0 ** n  # read psi and C, write psi per layer (complex64)
        row = {"workload": f"K{n} (seed {run.seed}) p={p} midpoint ramp D={run.delta_gamma}, complex64",
               "forward_ms": round(t_fwd, 3), "amp_layer_per_s": 2.0 ** n * p / (t_fwd * 1e-3),
               "algorithmic_gbs": round(alg / (t_fwd * 1e-3) / 1e9, 1),
               "algorithmic_hbm_frac": round(alg / (t_fwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "device_memory_gib": round(peak / 2 ** 30, 2), "exp_c": e, "r_exact": e / (sim.cmax / 10)}
        if grad:
            t_adj = float(np.median(ta))
            row.update({"forward_plus_adjoint_ms": round(t_adj, 3), "over_fwd": round(t_adj / t_fwd, 3)})
            log(f"huge_grad n={n}: forward {t_fwd:.1f} ms, forward+adjoint {t_adj:.1f} ms, "
                f"{peak / 2 ** 30:.0f} GiB")
            out["huge_grad"] = row
        else:
            row.update({"shots": run.shots, "sample_ms": round(float(np.median(tsm)), 3),
                        "r_shots": sim.shots_ratio(shots.cpu().numpy())})
            log(f"huge n={n}: forward {t_fwd:.1f} ms, {run.shots} shots {row['sample_ms']:.1f} ms, "
                f"{peak / 2 ** 30:.0f} GiB")
            out["huge"] = row
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return out


def noise_run(torch, workloads, stream, cpu: bool):
    """Noisy trajectories (Sec. II-C): throughput at n = 12, p = 10."""
    import numpy as np
    from paper_2604_26423_amd import Trajectories, linear_ramp, to_gate_angles
    from paper_2604_26423_amd import qs as Q
    b = workloads.NOISE_BENCH
    g, bb = linear_ramp(b.p, b.delta, b.delta, "midpoint")
    tzz, tx = to_gate_angles(g, bb, "paper")
    tr = Trajectories(b.weights(), "c64")
    dev = torch.device("cuda")
    exp_c = torch.empty(b.ntraj, dtype=torch.float64, device=dev)
    nerr = torch.empty(b.ntraj, dtype=torch.int32, device=dev)
    ts = []
    for _ in range(4):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        Q.qs_noise_run(tr.handle, tzz, tx, b.eps, b.seed, 0, b.ntraj, exp_c, None, nerr, None)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    t = float(np.median(ts[1:]))
    amp_layers = float(b.ntraj) * (1 << b.n) * b.p
    flops_per = 4 * b.n + 6  # tangent-form RX per qubit (2 complex FMAs) + the phase multiply
    achieved = amp_layers * flops_per / (t * 1e-3) / 1e12
    r = exp_c.cpu().numpy() / (tr.cmax / 10.0)
    ideal = tr.run(tzz, tx, 0.0, b.seed, 1)["exp_c"].cpu().numpy()[0] / (tr.cmax / 10.0)
    out = {"workload": f"K{b.n} (seed {b.seed}) p={b.p} midpoint ramp D={b.delta}, eps={b.eps} after every "
                       f"RZZ gate, {b.ntraj} trajectories, complex64",
           "ms": round(t, 3), "trajectories_per_s": b.ntraj / (t * 1e-3),
           "amp_layer_per_s": amp_layers / (t * 1e-3),
           "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / FP32_VECTOR_TFLOPS, 4), "flops_per_amp_layer": flops_per,
                        "traffic": None},
           "r_noisy": float(r.mean()), "r_noisy_sem": float(r.std(ddof=1) / np.sqrt(len(r))),
           "r_ideal": float(ideal), "r_random": tr.random_ratio(),
           "mean_errors_per_trajectory": float(nerr.double().mean().item())}
    tr.close()
    log(f"noise: {b.ntraj} trajectories n={b.n} p={b.p} in {t:.2f} ms "
        f"({out['amp_layer_per_s']:.3g} amp-layer/s, {achieved:.1f} TFLOP/s)")
    if cpu:
        import oracle
        w = b.weights()
        k = 4
        t0 = time.perf_counter()
        for i in range(k):
            oracle.noisy_trajectory(b.n, w, tzz, tx, b.eps, b.seed, i)
        tc = time.perf_counter() - t0
        out["cpu_oracle"] = {"trajectories_per_s": k / tc, "amp_layer_per_s": k * (1 << b.n) * b.p / tc,
                             "cores": oracle.num_threads(), "kind": "oracle",
                             "sample": f"{k} trajectories of the same workload, gate by gate, complex128"}
    torch.cuda.empty_cache()
    return out


def sweep30(torch, workloads, Simulator, linear_ramp, to_gate_angles, stream):
    """Forward and forward+adjoint at n = 30 for each depth of the sweep."""
    rows = []
    sim = None
    for run in workloads.SWEEP30:
        if sim is None:
            sim = Simulator(run.weights(), "c64")
        g, b = linear_ramp(run.p, run.delta_gamma, run.delta_beta, "midpoint")
        tzz, tx = to_gate_angles(g, b, "paper")
        tf, ta = [], []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            e, _ = sim.forward(tzz, tx)
            e1.record(stream)
            sim.adjoint(tzz, tx)
            e2.record(stream)
            torch.cuda.synchronize()
            tf.append(e0.elapsed_time(e1))
            ta.append(e1.elapsed_time(e2))
        t_fwd, t_adj = min(tf[1:]), min(ta[1:])
        row = {"p": run.p, "forward_ms": round(t_fwd, 3), "forward_plus_adjoint_ms": round(t_adj, 3),
               "amp_layer_per_s": 2.0 ** run.n * run.p / (t_fwd * 1e-3), "r_exact": e / (sim.cmax / 10)}
        log(f"sweep30 p={run.p}: forward {t_fwd:.1f} ms, forward+adjoint {t_adj:.1f} ms, r {row['r_exact']:.6f}")
        rows.append(row)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--shots", type=int, default=10000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-c128", action="store_true", help="skip the complex128 comparison")
    ap.add_argument("--cpu-n", type=int, default=27, help="qubits of the CPU oracle sample")
    ap.add_argument("--cpu-n1", type=int, default=22, help="qubits of the single-thread CPU oracle sample")
    ap.add_argument("--no-sweep30", action="store_true", help="skip the 30-qubit depth sweep")
    ap.add_argument("--no-sym", action="store_true", help="skip the complement-symmetric layout run")
    ap.add_argument("--no-store", action="store_true", help="skip the store-mode (checkpointed) adjoint run")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-circuit batched forward+adjoint")
    ap.add_argument("--no-huge", action="store_true", help="skip the K34 forward and the K33 forward+adjoint")
    ap.add_argument("--no-noise", action="store_true", help="skip the noisy-trajectory runs")
    ap.add_argument("--noise-only", action="store_true",
                    help="run only the noisy-trajectory section and print its JSON object")
    ap.add_argument("--no-window", action="store_true", help="skip the mixer-window butterfly / matrix-core probe")
    ap.add_argument("--window-only", action="store_true",
                    help="run only the mixer-window butterfly / matrix-core probe and print its JSON object")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py runs on one GPU only: the simulator does not shard the state across GPUs "
            "(rerun with --gpus 1)")
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2604_26423_amd import Simulator, linear_ramp, to_gate_angles
    from paper_2604_26423_amd import qs as Q

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.noise_only:
        print(json.dumps({"noise": noise_run(torch, workloads, torch.cuda.current_stream(), not args.no_cpu)}))
        return
    if args.window_only:
        print(json.dumps({"window_probe": window_microbench(torch, Q)}))
        return
    run = workloads.LARGE
    n, p = args.n, args.p
    w = workloads.complete_graph_tenths(n, run.seed)
    g, b = linear_ramp(p, run.delta_gamma, run.delta_beta, "midpoint")
    tzz, tx = to_gate_angles(g, b, "paper")
    stream = torch.cuda.current_stream()

    ceiling = device_ceiling(torch, Q)
    log("device ceilings (probe kernels, 4 GiB): " +
        ", ".join(f"{k} {ceiling[k]['gbs']} GB/s" for k in ("read", "write", "copy", "update")))
    log(f"setup: n={n} p={p} c64 state {2 ** n * 8 / 2 ** 30:.0f} GiB + diag {2 ** n * 4 / 2 ** 30:.0f} GiB")
    sim = Simulator(w, "c64")
    sim.lam = torch.empty_like(sim.psi)
    lam_bytes = sim.lam.numel() * sim.lam.element_size()

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def step():
        e0 = ev()
        W, cmax = Q.qs_cost_diagonal(n, w, sim.diag, stream)
        e1 = ev()
        exp_c, nrm = sim.forward(tzz, tx)
        e2 = ev()
        shots = sim.sample(args.shots, run.seed, on_device=True)
        e3 = ev()
        ea, gzz, gx = Q.qs_adjoint_grad(sim.handle, sim.diag, sim.w_total, tzz, tx, sim.lam, lam_bytes)
        e4 = ev()
        torch.cuda.synchronize()
        t = [e0.elapsed_time(e1), e1.elapsed_time(e2), e2.elapsed_time(e3), e3.elapsed_time(e4),
             e0.elapsed_time(e4)]
        return t, dict(exp_c=exp_c, norm=nrm, cmax=cmax, w_total=W, grad_zz=list(gzz), grad_x=list(gx),
                       exp_c_adj=ea, shots=shots)

    for i in range(args.warmup):
        t, _ = step()
        log(f"warmup {i}: step {t[4]:.1f} ms (diag {t[0]:.1f}, fwd {t[1]:.1f}, sample {t[2]:.1f}, "
            f"fwd+adjoint {t[3]:.1f})")

    torch.cuda.synchronize()
    Q.qs_profile(sim.handle, True)
    times = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        t, res = step()
        times.append(t)
        log(f"step {i}: {t[4]:.1f} ms (diag {t[0]:.1f}, fwd {t[1]:.1f}, sample {t[2]:.1f}, "
            f"fwd+adjoint {t[3]:.1f})")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    prof = {Q.KIND_NAMES[k]: Q.qs_profile_read(sim.handle, k) for k in range(Q.QS_KIND_COUNT)}
    Q.qs_profile(sim.handle, False)

    T = np.array(times)
    # medians over the timed steps (the means are reported beside them)
    t_diag, t_fwd, t_smp, t_adj, t_step = np.median(T, axis=0)
    m_diag, m_fwd, m_smp, m_adj, m_step = T.mean(axis=0)
    r_exact = res["exp_c"] / (res["cmax"] / 10)
    shots_host = res["shots"].cpu().numpy()
    r_shots = sim.shots_ratio(shots_host)

    # dominant kernel (symbol) by total event time inside the timed steps;
    # kinds that share a kernel are combined
    by_kernel = {}
    for kind, (cnt, ms, by) in prof.items():
        k = Q.KIND_KERNEL[kind]
        c0, m0, b0 = by_kernel.get(k, (0, 0.0, 0.0))
        by_kernel[k] = (c0 + cnt, m0 + ms, b0 + by)
    dom = max(by_kernel, key=lambda k: by_kernel[k][1])
    launches, ms, by = by_kernel[dom]
    avg_ms = ms / max(launches, 1)
    dim = 2.0 ** n
    # Algorithmic bytes per amplitude and layer (complex64): a forward layer
    # must read psi and C and write psi (20 B); a reverse layer must read psi,
    # lambda and C and write psi and lambda (36 B).  A launch of a kernel
    # covers the layers of its sweep divided by the sweep's launches.
    n_fwd = Q.qs_adjoint_ckpt_bytes(sim.handle, p) // Q.qs_state_bytes(n, Q.QS_C64) + 2  # tile passes of a forward
    alg_layer = {"pass_kernel": (20.0, n_fwd), "adjoint_kernel<reverse>": (36.0, n_fwd),
                 "adjoint_kernel<turnaround>": (36.0, n_fwd)}
    per_amp, cover = alg_layer.get(dom, (20.0, n_fwd))
    alg_per_launch = per_amp * dim * p / cover
    achieved = alg_per_launch / (avg_ms * 1e-3) / 1e9
    design_bpl = by / max(launches, 1)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
                "launches": launches, "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": alg_per_launch,
                "algorithmic_bytes_per_amp_layer": per_amp, "launches_per_sweep": cover,
                "design_bytes_per_launch": design_bpl,
                "design_bytes_gbs": round(design_bpl / (avg_ms * 1e-3) / 1e9, 1),
                "copy_ceiling_gbs": ceiling["copy_ceiling_gbs"],
                "design_frac_of_copy_ceiling": round(design_bpl / (avg_ms * 1e-3) / 1e9 /
                                                     ceiling["copy_ceiling_gbs"], 4)}
    per_kind = {k: {"launches": v[0], "ms_total": round(v[1], 3),
                    "design_gbs": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
                for k, v in prof.items() if v[0] > 0}

    # algorithmic bytes of the forward: read C and psi, write psi once per layer
    alg_fwd = dim * p * (4 + 8 + 8)
    out = {
        "metric": "amp-layer updates/s (forward, n=32 p=3 complex64)",
        "value": dim * p / (t_fwd * 1e-3),
        "unit": "amp-layer updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(float(t_step), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"K{n} weighted complete graph (seed {run.seed}, weights 1..10 tenths), "
                               f"LR-QAOA p={p}, midpoint ramp D=0.6, complex64, {args.shots} shots, "
                               f"forward + adjoint gradient",
                   "n": n, "p": p, "precision": "c64", "shots": args.shots, "convention": "paper"},
        "breakdown_ms": {"cost_diagonal": round(float(t_diag), 3), "forward_with_readout": round(float(t_fwd), 3),
                         "sample": round(float(t_smp), 3), "forward_plus_adjoint": round(float(t_adj), 3),
                         "statistic": "median over the timed steps"},
        "breakdown_ms_mean": {"cost_diagonal": round(float(m_diag), 3), "forward_with_readout": round(float(m_fwd), 3),
                              "sample": round(float(m_smp), 3), "forward_plus_adjoint": round(float(m_adj), 3),
                              "step": round(float(m_step), 3)},
        "fwd_adjoint_over_fwd": round(float(t_adj / t_fwd), 3),
        "device_ceiling": ceiling,
        "forward_algorithmic_hbm_frac": round(alg_fwd / (t_fwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "kernels": per_kind,
        "results": {"exp_c": res["exp_c"], "norm_minus_1": res["norm"] - 1, "r_exact": r_exact,
                    "r_shots": r_shots, "cmax_tenths": res["cmax"], "w_total_tenths": res["w_total"],
                    "grad_theta_zz": res["grad_zz"], "grad_theta_x": res["grad_x"]},
        "wall_s_timed": round(wall, 3),
    }

    if not args.no_store:
        # the store mode of the adjoint: per-pass checkpoints instead of
        # undoing the passes on psi (5 states of 32 GiB at n=32, p=3)
        need = Q.qs_adjoint_ckpt_bytes(sim.handle, p)
        torch.cuda.empty_cache()
        free = torch.cuda.mem_get_info()[0]
        if free < need + (4 << 30):
            out["store_mode"] = {"skipped": f"needs {need / 2 ** 30:.0f} GiB of checkpoints, "
                                            f"{free / 2 ** 30:.0f} GiB free"}
        else:
            ck = torch.empty(need, dtype=torch.uint8, device="cuda")
            ts = []
            for i in range(3):
                a = ev()
                es, szz, sx = Q.qs_adjoint_grad_store(sim.handle, sim.diag, sim.w_total, tzz, tx, ck, need,
                                                      sim.lam, lam_bytes)
                bb = ev()
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(bb))
                log(f"store-mode forward+adjoint {i}: {ts[-1]:.1f} ms")
            del ck
            torch.cuda.empty_cache()
            t_st = float(np.median(ts[1:]))
            uzz, ux = np.array(res["grad_zz"]), np.array(res["grad_x"])
            scale = max(np.abs(uzz).max(), np.abs(ux).max())
            out["store_mode"] = {"forward_plus_adjoint_ms": round(t_st, 3), "over_fwd": round(t_st / float(t_fwd), 3),
                                 "checkpoint_gib": need / 2 ** 30,
                                 "grad_rel_diff_vs_uncompute": max(np.abs(szz - uzz).max(),
                                                                   np.abs(sx - ux).max()) / scale,
                                 "exp_c_rel_diff": abs(es - res["exp_c"]) / res["exp_c"]}

    if not args.no_c128:
        # the same forward and gradient in complex128 (64 GiB state, 64 GiB
        # adjoint vector), sharing the diagonal: its time, and the complex64
        # errors against it
        sim.lam = None
        torch.cuda.empty_cache()
        log("c128 comparison: allocating a 64 GiB state")
        psi128 = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
        h = Q.qs_alloc(n, Q.QS_C128, psi128, psi128.numel() * 16, stream)
        tt = []
        for i in range(3):
            a = ev()
            e128, _ = Q.qs_forward(h, sim.diag, sim.w_total, tzz, tx)
            bb = ev()
            torch.cuda.synchronize()
            tt.append(a.elapsed_time(bb))
            log(f"c128 forward {i}: {tt[-1]:.1f} ms")
        lam128 = torch.empty_like(psi128)
        a = ev()
        ea128, gzz128, gx128 = Q.qs_adjoint_grad(h, sim.diag, sim.w_total, tzz, tx, lam128, lam128.numel() * 16)
        bb = ev()
        torch.cuda.synchronize()
        t128a = a.elapsed_time(bb)
        Q.qs_free(h)
        del psi128, lam128
        torch.cuda.empty_cache()
        t128 = float(np.median(tt[1:]))
        gz, gxx = np.array(res["grad_zz"]), np.array(res["grad_x"])
        gscale = max(np.abs(gzz128).max(), np.abs(gx128).max())
        out["c128"] = {"forward_ms": round(t128, 3), "amp_layer_per_s": dim * p / (t128 * 1e-3),
                       "c64_speedup": round(t128 / float(t_fwd), 3), "forward_plus_adjoint_ms": round(t128a, 3),
                       "exp_c": e128, "c64_exp_c_rel_err": abs(res["exp_c"] - e128) / e128,
                       "c64_grad_abs_err": float(max(np.abs(gz - gzz128).max(), np.abs(gxx - gx128).max())),
                       "c64_grad_rel_err": float(max(np.abs(gz - gzz128).max(), np.abs(gxx - gx128).max()) / gscale),
                       "grad_theta_zz": list(gzz128), "grad_theta_x": list(gx128)}
        log(f"c128: forward {t128:.1f} ms, forward+adjoint {t128a:.1f} ms; complex64 <C> error "
            f"{out['c128']['c64_exp_c_rel_err']:.2e}, gradient error {out['c128']['c64_grad_rel_err']:.2e}")

    # the literal reading of the gate angles (same kernels, other angles)
    # exact cut-value distribution of the final state (one pass over psi and C)
    sim.forward(tzz, tx)
    nb = int(res["w_total"]) + 1
    hist = torch.empty(nb, dtype=torch.int64, device="cuda")
    th = []
    for _ in range(4):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        Q.qs_cost_histogram(sim.handle, sim.diag, nb, hist)
        e1.record(stream)
        torch.cuda.synchronize()
        th.append(e0.elapsed_time(e1))
    t_h = float(np.median(th[1:]))
    mass = hist.cpu().numpy().view(np.uint64).astype(np.float64) / 2.0 ** 62
    hgbs = dim * 12 / (t_h * 1e-3) / 1e9  # algorithmic: read psi (8 B) and C (4 B) per amplitude
    out["histogram"] = {"ms": round(t_h, 3), "bins": nb, "gbs": round(hgbs, 1),
                        "roofline": {"bound": "hbm", "achieved": round(hgbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": round(hgbs / HBM_PEAK_GBS, 4), "traffic": None},
                        "total_probability": float(mass.sum()),
                        "exp_c_from_histogram": float((mass * np.arange(nb)).sum() / mass.sum() / 10)}
    log(f"histogram: {nb} bins in {t_h:.2f} ms")

    tzz_l, tx_l = to_gate_angles(g, b, "literal")
    e_lit, _ = sim.forward(tzz_l, tx_l)
    out["results"]["r_exact_literal_convention"] = e_lit / (res["cmax"] / 10)
    sim.close()
    del sim
    torch.cuda.empty_cache()

    if not args.no_sym:
        out["symmetric"] = symmetric_run(torch, Simulator, w, tzz, tx, res["exp_c"], stream)

    if not args.no_batch:
        out["batch"] = batch_run(torch, workloads, stream, not args.no_cpu)

    if not args.no_huge:
        out.update(huge_run(torch, workloads, Simulator, linear_ramp, to_gate_angles, stream))

    if not args.no_window:
        out["window_probe"] = window_microbench(torch, Q)

    if not args.no_noise:
        out["noise"] = noise_run(torch, workloads, stream, not args.no_cpu)

    if not args.no_sweep30:
        out["sweep30"] = sweep30(torch, workloads, Simulator, linear_ramp, to_gate_angles, stream)

    if not args.no_cpu:
        import oracle
        nc = args.cpu_n
        wc = workloads.complete_graph_tenths(nc, run.seed)
        log(f"cpu baseline: oracle, gate-by-gate complex128, n={nc} p={p} on {oracle.num_threads()} threads")
        t0 = time.perf_counter()
        psi_c = oracle.simulate(nc, wc, tzz, tx, mode=0)
        tc = time.perf_counter() - t0
        host = host_info()
        n1 = args.cpu_n1
        t1 = single_thread_oracle(n1, run.seed, tzz, tx)
        out["cpu_baseline"] = {"value": 2.0 ** nc * p / tc, "unit": "amp-layer updates/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"K{nc} (seed {run.seed}) p={p} forward, gate by gate "
                                         f"(n(n-1)/2 RZZ + n RX passes per layer), complex128, {tc:.1f} s",
                               "seconds": round(tc, 2), **host,
                               "single_thread": {"value": 2.0 ** n1 * p / t1, "unit": "amp-layer updates/s",
                                                 "seconds": round(t1, 2),
                                                 "sample": f"K{n1} (seed {run.seed}) p={p} forward, one thread"}}
        log(f"cpu baseline: {tc:.1f} s")
        if "histogram" in out:
            dg = oracle.cost_diagonal(nc, wc)
            t0 = time.perf_counter()
            oracle.cost_histogram(psi_c, dg, int(dg.max()) + 1)
            th = time.perf_counter() - t0
            out["histogram"]["cpu_oracle"] = {"amplitudes_per_s": 2.0 ** nc / th, "kind": "oracle",
                                              "sample": f"K{nc} final state of the CPU baseline, {th:.2f} s"}
        del psi_c

    print(json.dumps(out))


if __name__ == "__main__":
    main()
