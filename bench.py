#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

Step (timed K times after W warm-ups): one pass of every single-GPU step of
the path over a seeded random 30-qubit complex64 state (8 GiB, resident in
HBM):
  * a Haar U(2) on every target qubit 0..29 (eq. (1), k = 1);
  * controlled gates CNOT(0->29), CZ(3,17), CRZ(29->0);
  * dense Haar U(4) / U(8) on low, mixed and high target sets;
  * permutation and diagonal gates X(29), SWAP(0,29), Z(5), a phase on 12;
  * fused dense 4- and 5-qubit blocks (matrix cores) on low, high and mixed
    targets;
  * the open-chain transverse-field Ising energy and the norm (each counted as
    one read of the state, the least any implementation needs).
value = algorithmic bytes of the step (each touched amplitude read and
written once; read-only passes counted once) / measured time.

Side measurements (reported, not part of `value`): per-target GB/s of the
single-qubit sweep for complex64 and complex128, the adjoint gradient of the
hardware-efficient ansatz (n = 20, 8 layers) in gradients/s against plain
parameter shift on the same GPU, the roofline of the dominant kernel timed
with HIP events, and the CPU oracle on a bounded sample (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitude GB/s vs HBM peak at 30q; adjoint grads/s vs parameter-shift"
HBM_PEAK_GBS = 8000.0


def step_ops(n, rng, W):
    ops = [W.Op("matrix", (t,), matrix=W.haar_unitary(rng, 2)) for t in range(n)]
    ops += [W.Op("x", (n - 1,), controls=(0,)), W.Op("z", (17,), controls=(3,)),
            W.Op("rz", (0,), controls=(n - 1,), param=0)]
    for t in [(0, 1), (1, n - 1), (n - 2, n - 1), (0, 1, 2), (2, n // 2, n - 1),
              (n - 3, n - 2, n - 1)]:
        ops.append(W.Op("matrix", t, matrix=W.haar_unitary(rng, 2 ** len(t))))
    ops += [W.Op("x", (n - 1,)), W.Op("swap", (0, n - 1)), W.Op("z", (5,)),
            W.Op("matrix", (12,), matrix=__import__("numpy").diag([1, 1j]).astype(complex))]
    for t in [(0, 1, 2, 3), (n - 4, n - 3, n - 2, n - 1), (0, 1, 2, 3, 4),
              (n - 5, n - 4, n - 3, n - 2, n - 1), (0, 9, 15, 22, n - 1)]:
        ops.append(W.Op("matrix", t, matrix=W.haar_unitary(rng, 2 ** len(t))))
    return W.Circuit(n, ops, 1)


def recorded_traffic():
    """HBM bytes per dispatch of the dominant kernel from the committed
    rocprofv3 counter summary, or None once the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_dense_sweep_n30_c64_hbm_counters.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic-record:"):
            rec = dict(kv.split("=", 1) for kv in line.split()[1:])
    if not rec:
        return None
    src = open(os.path.join(ROOT, rec["src"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["src_sha256"]:
        return None
    return (float(rec["fetch_kib"]) * float(rec["fetch_factor"]) +
            float(rec["write_kib"]) * float(rec["write_factor"])) * 1024.0


def event_time(fn, reps, stream):
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_gate_rates(n, targets, reps=1):
    """The oracle (as written: complex128, out of place, OpenMP over output
    indices) applying a Haar U(2) on each target of a seeded n-qubit state;
    returns {target: GB/s} counting 2 x 16 B per amplitude like the GPU
    figure, and the threads the oracle used."""
    import numpy as np

    import oracle
    import workloads as W
    rng = np.random.default_rng(1000)
    psi = oracle.random_state(n, 7)
    out = {}
    for t in targets:
        G = W.haar_unitary(rng, 2)
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            res = oracle.apply(psi, (t,), (), G)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
            del res
        out[t] = 2.0 * 16 * (1 << n) / best / 1e9
    return out, int(oracle.lib().orc_threads())


def cpu_baseline():
    """The CPU oracle (never tuned) on a bounded sample of the headline sweep:
    one Haar U(2) gate at every target 0..29 of a seeded 30-qubit complex128
    state on every host thread (the GPU's per-target sweep, one gate each),
    and at targets 0, 15 and 27 of a 28-qubit state on one thread (a child
    process with OMP_NUM_THREADS=1; one thread at 30 qubits would take ~10 s
    per gate).  value = mean all-thread GB/s over the 30 targets."""
    import subprocess
    n = 30
    t0 = time.perf_counter()
    rates, threads = oracle_gate_rates(n, tuple(range(n)))
    t_all = time.perf_counter() - t0
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import json, sys; sys.path.insert(0, %r); import bench; r, th = bench.oracle_gate_rates(28, (0, 15, 27)); "
            "print(json.dumps({'rates': r, 'threads': th}))" % ROOT)
    t1 = time.perf_counter()
    one = None
    try:
        p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        if p.returncode == 0:
            one = json.loads(p.stdout.strip().splitlines()[-1])
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        one = None
    t_one = time.perf_counter() - t1
    value = sum(rates.values()) / len(rates)
    res = {"value": round(value, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": "oracle eq.(1), complex128, out of place: one Haar U(2) gate at each target 0..29 of "
                     "a seeded 30-qubit state (16 GiB in + 16 GiB out per gate) on %d threads (%.1f s incl. "
                     "state set-up); GB/s counts 2 x 16 B per amplitude like the GPU figure" % (threads, t_all),
           "seconds": round(t_all, 1),
           "per_target_gbs": [round(rates[t], 2) for t in range(n)],
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "affinity_cpus": len(os.sched_getaffinity(0)),
           "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}
    if one:
        r1 = {str(k): round(v, 3) for k, v in one["rates"].items()}
        res["one_thread"] = {"n": 28, "threads": one["threads"], "per_target_gbs": r1,
                             "value": round(sum(one["rates"].values()) / len(r1), 3),
                             "seconds": round(t_one, 1)}
    return res


def profile_kernels():
    """Short run for rocprofv3 counter passes: a 4 GiB torch copy (the
    calibration kernel of known traffic) twice, then the single-qubit sweep
    (n = 30, complex64, target 15) ten times."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2202_07017_amd import qsv
    dev = torch.device("cuda:0")
    src = torch.empty(1 << 29, dtype=torch.float64, device=dev)
    src.fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    del src, dst
    psi = torch.empty(1 << 30, dtype=torch.complex64, device=dev)
    qsv.qsv_init_random(psi, 5)
    G = W.haar_unitary(np.random.default_rng(1), 2)
    for _ in range(10):
        qsv.qsv_apply_gate(psi, (15,), (), G)
    torch.cuda.synchronize()
    print("profile run done: 2 x 4 GiB copy, 10 x single-qubit sweep n=30 c64 t=15", flush=True)


def profile_circuits():
    """Short run for rocprofv3 counter passes over the plan kernels: a 4 GiB
    torch copy (calibration) twice, then the QFT at n = 30 complex64 fused to
    k = 5 (matrix-core blocks, diagonal runs, the qubit permutation pass) and
    unfused (runs with gates in their sweeps), twice each."""
    import torch

    import workloads as W
    from paper_2202_07017_amd import qsv
    dev = torch.device("cuda:0")
    src = torch.empty(1 << 29, dtype=torch.float64, device=dev)
    src.fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    del src, dst
    n = 30
    psi = torch.empty(1 << n, dtype=torch.complex64, device=dev)
    qsv.qsv_init_random(psi, 5)
    for fuse in (5, 1):
        plan = qsv.Plan(W.qft(n), qsv.C64, fuse)
        for _ in range(2):
            plan.run(psi)
    torch.cuda.synchronize()
    print("profile run done: 2 x 4 GiB copy, QFT n=30 c64 fused k=5 and unfused, 2 runs each", flush=True)


def profile_mfma():
    """Short run for the matrix-core counters: fused dense blocks of k = 4 and
    k = 5 qubits (Haar unitaries) on a 30-qubit state, complex64 then
    complex128, five launches each on low and on spread targets."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2202_07017_amd import qsv
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(1005)
    n = 30
    for dt in (torch.complex64, torch.complex128):
        psi = torch.empty(1 << n, dtype=dt, device=dev)
        qsv.qsv_init_random(psi, 5)
        for t in [(0, 1, 2, 3), (0, 1, 2, 3, 4), (3, 11, 19, 27), (2, 9, 15, 22, 29)]:
            G = W.haar_unitary(rng, 2 ** len(t))
            for _ in range(5):
                qsv.qsv_apply_gate(psi, t, (), G)
        torch.cuda.synchronize()
        del psi
        torch.cuda.empty_cache()
    print("profile run done: k = 4, 5 fused blocks, n=30, c64 and c128, 5 launches per target set",
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--skip-side", action="store_true", help="only the timed step")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only the dominant kernel and a copy of known size (counter runs)")
    ap.add_argument("--profile-circuits", action="store_true",
                    help="short run for counter passes over the plan kernels (QFT n=30 c64)")
    ap.add_argument("--profile-mfma", action="store_true",
                    help="only fused k = 4, 5 blocks (matrix-core counter runs)")
    ap.add_argument("--legs", default="",
                    help="comma list of side legs to run alone (adjoint, adjoint26, batched, configs, expect, measure, circuits): profiling runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path runs on a single MI355X and the library has no "
              "multi-GPU mode (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.profile_kernels:
        profile_kernels()
        return
    if args.profile_circuits:
        profile_circuits()
        return
    if args.profile_mfma:
        profile_mfma()
        return
    if args.legs:
        import numpy as np
        import torch

        import workloads as W
        from paper_2202_07017_amd import qsv
        dev = torch.device("cuda:0")
        out = {}
        legs = set(args.legs.split(","))
        if "adjoint" in legs:
            out["adjoint"] = adjoint_leg(qsv, W, torch, np, dev)
        if "adjoint26" in legs:
            out["adjoint_n26"] = adjoint_leg_large(qsv, W, torch, np, dev)
        if "batched" in legs:
            out["batched"] = batched_leg(qsv, W, torch, np, dev)
        if "configs" in legs:
            out["configs"] = configs_leg(qsv, W, torch, np, dev, torch.cuda.current_stream())
        if "expect" in legs:
            out["expectation"] = expectation_leg(qsv, W, torch, np, dev, torch.cuda.current_stream())
        if "measure" in legs:
            out["measure"] = measure_leg(qsv, W, torch, np, dev, torch.cuda.current_stream())
        if "circuits" in legs:
            out["qft_trotter"] = qft_trotter_leg(qsv, W, torch, np, dev, torch.cuda.current_stream())
        print(json.dumps(out), flush=True)
        return

    import numpy as np
    import torch

    import workloads as W
    from paper_2202_07017_amd import qsv

    n = args.n
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(1002)
    circ = step_ops(n, rng, W)
    plan = qsv.Plan(circ, qsv.C64, 1, params_host=np.array([1.234]))
    nl, plan_bytes, plan_flops = plan.info()
    H = qsv.PauliSum(W.tfim_chain(n))
    S = 8
    # algorithmic bytes: every gate reads and writes each amplitude it touches
    # once; the energy and the norm each read the state once
    step_bytes = plan_bytes + S * (1 << n) + S * (1 << n)
    psi = torch.empty(1 << n, dtype=torch.complex64, device=dev)
    qsv.qsv_init_random(psi, 1002)
    e_out = torch.empty(2, dtype=torch.float64, device=dev)
    n_out = torch.empty(1, dtype=torch.float64, device=dev)

    def step():
        plan.run(psi)
        qsv.qsv_expectation(psi, H, e_out)
        qsv.qsv_norm2(psi, n_out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = elapsed / args.steps * 1e3
    value = step_bytes * args.steps / elapsed / 1e9
    norm = float(n_out.cpu()[0])

    # Dominant kernel: the single-qubit sweep (30 of the step's launches),
    # timed with HIP events on the stream it is launched on.
    G = W.haar_unitary(rng, 2)
    reps = 20
    sweep_bytes = 2.0 * S * (1 << n)
    avg = event_time(lambda: qsv.qsv_apply_gate(psi, (15,), (), G), reps, stream)
    roof = {"bound": "hbm", "achieved": round(sweep_bytes / avg / 1e9, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(sweep_bytes / avg / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(), "kernel": "k_dense<float,1,W2> (single-qubit sweep, target 15)",
            "avg_launch_ms": round(avg * 1e3, 4)}
    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded random state, Haar-random gates)",
           "config": {"workload": "n=30 complex64 gate sweeps + TFIM energy + norm", "n": n,
                      "state": "complex64",
                      "launches_per_step": nl + qsv.expectation_launches(H, n, qsv.C64) + 2,
                      "step_bytes": step_bytes, "hbm_frac": round(value / HBM_PEAK_GBS, 4),
                      "norm_after": norm},
           "roofline": roof}

    if not args.skip_side:
        per = {}
        for name, dt in [("c64", torch.complex64), ("c128", torch.complex128)]:
            del psi
            torch.cuda.empty_cache()
            psi = torch.empty(1 << n, dtype=dt, device=dev)
            qsv.qsv_init_random(psi, 5)
            Sb = 8 if name == "c64" else 16
            row = []
            for t in range(n):
                a = event_time(lambda: qsv.qsv_apply_gate(psi, (t,), (), G), 5, stream)
                row.append(round(2.0 * Sb * (1 << n) / a / 1e9, 1))
            per[name] = row
        out["per_target_gbs"] = per
        del psi
        torch.cuda.empty_cache()
        out["adjoint"] = adjoint_leg(qsv, W, torch, np, dev)
        out["adjoint_n26"] = adjoint_leg_large(qsv, W, torch, np, dev)
        out["batched"] = batched_leg(qsv, W, torch, np, dev)
        out["configs"] = configs_leg(qsv, W, torch, np, dev, stream)
        out["expectation"] = expectation_leg(qsv, W, torch, np, dev, stream)
        out["measure"] = measure_leg(qsv, W, torch, np, dev, stream)
        out["qft_trotter"] = qft_trotter_leg(qsv, W, torch, np, dev, stream)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def expectation_leg(qsv, W, torch, np, dev, stream, n=30):
    """<psi|H|psi> on a seeded 30-qubit state for the open-chain TFIM (h = 1),
    the XXZ chain (Delta = 0.5) and 64 random Pauli strings: ms per
    evaluation, kernel launches, and GB/s counting one read of the state (the
    least any implementation needs)."""
    res = {}
    hams = (("tfim", W.tfim_chain(n)), ("xxz", W.xxz_chain(n, 0.5)), ("random64", W.random_pauli_sum(n, 64, 77)))
    for name, dt, code, S in (("c64", torch.complex64, qsv.C64, 8), ("c128", torch.complex128, qsv.C128, 16)):
        psi = torch.empty(1 << n, dtype=dt, device=dev)
        qsv.qsv_init_random(psi, 4004)
        out = torch.empty(2, dtype=torch.float64, device=dev)
        for tag, h in hams:
            H = qsv.PauliSum(h)
            qsv.qsv_expectation(psi, H, out)
            a = event_time(lambda: qsv.qsv_expectation(psi, H, out), 5, stream)
            res["%s_n%d_%s" % (tag, n, name)] = {
                "ms": round(a * 1e3, 3), "launches": qsv.expectation_launches(H, n, code),
                "terms": int(len(h.coeff)),
                "gbs_one_read": round(S * (1 << n) / a / 1e9, 1)}
        del psi
        torch.cuda.empty_cache()
    return res


def measure_leg(qsv, W, torch, np, dev, stream, n=30, shots=1 << 20):
    """Simulated measurement on the seeded 30-qubit state: marginal
    probabilities of 1, 10 (lowest / highest) and 20 qubits (GB/s = one read
    of the state / time), and shot sampling: the prefix pass alone (one shot)
    and 2^20 shots, giving the pass's GB/s and the per-shot rate, the
    frequencies of those shots over 10 qubits, and the collapse sweep onto one
    outcome of 3 qubits (GB/s = read + write of the state / time)."""
    res = {}
    u = torch.from_numpy(W.uniforms(shots, 2024)).to(dev)
    for name, dt, S in (("c64", torch.complex64, 8), ("c128", torch.complex128, 16)):
        psi = torch.empty(1 << n, dtype=dt, device=dev)
        qsv.qsv_init_random(psi, 2024)
        out = torch.empty(1 << 20, dtype=torch.float64, device=dev)
        row = {}
        for tag, qs in (("q15", [15]), ("low10", list(range(9, -1, -1))),
                        ("high10", list(range(29, 19, -1))),
                        ("spread20", list(range(0, 30, 3)) + list(range(1, 30, 3)))):
            a = event_time(lambda: qsv.qsv_probabilities(psi, qs, out=out), 5, stream)
            row["probabilities_" + tag + "_gbs"] = round(S * (1 << n) / a / 1e9, 1)
        samples = torch.empty(shots, dtype=torch.int64, device=dev)
        t1 = event_time(lambda: qsv.qsv_sample(psi, u[:1], out=samples[:1]), 5, stream)
        tn = event_time(lambda: qsv.qsv_sample(psi, u, out=samples), 5, stream)
        row["sample_prefix_pass_gbs"] = round(S * (1 << n) / t1 / 1e9, 1)
        row["sample_%d_shots_ms" % shots] = round(tn * 1e3, 3)
        row["shots_per_s_after_pass"] = round(shots / max(tn - t1, 1e-9), 1)
        cnt = torch.empty(1 << 10, dtype=torch.int64, device=dev)
        tf = event_time(lambda: qsv.qsv_frequencies(samples, n, list(range(9, -1, -1)), out=cnt), 5, stream)
        row["frequencies_10q_%d_shots_ms" % shots] = round(tf * 1e3, 3)
        pr = qsv.qsv_probabilities(psi, [29, 0, 15])
        tc = event_time(lambda: qsv.qsv_collapse(psi, [29, 0, 15], 5, pr[5:6]), 3, stream)
        row["collapse_gbs"] = round(2.0 * S * (1 << n) / tc / 1e9, 1)
        res[name] = row
        del psi, out, samples
        torch.cuda.empty_cache()
    return res


def qft_trotter_leg(qsv, W, torch, np, dev, stream, n=30):
    """Two more workloads at n = 30 as whole plans: the QFT (Hadamards,
    controlled phases, swaps) and one symmetric Trotter step of the TFIM
    (h = 1), each unfused and fused to k = 5; ms per run, launches, and GB/s
    and TFLOP/s of the plan's algorithmic bytes and flops."""
    res = {}
    for name, dt, code in (("c64", torch.complex64, qsv.C64), ("c128", torch.complex128, qsv.C128)):
        psi = torch.empty(1 << n, dtype=dt, device=dev)
        qsv.qsv_init_random(psi, 3003)
        for tag, make in (("qft", lambda k: qsv.Plan(W.qft(n), code, k)),
                          ("trotter_tfim_order2", lambda k: qsv.TrotterPlan(W.tfim_chain(n), 0.05, 1, 2,
                                                                            code, k))):
            for k in (1, 5):
                plan = make(k)
                nl, b, f = plan.info()
                plan.run(psi)
                a = event_time(lambda: plan.run(psi), 2, stream)
                res["%s_n%d_%s_fuse%d" % (tag, n, name, k)] = {
                    "ms": round(a * 1e3, 3), "launches": nl, "gbs": round(b / a / 1e9, 1),
                    "hbm_frac": round(b / a / 1e9 / HBM_PEAK_GBS, 4), "tflops": round(f / a / 1e12, 2)}
                del plan
        del psi
        torch.cuda.empty_cache()
    return res


def configs_leg(qsv, W, torch, np, dev, stream):
    """The seeded random circuits of the workload list, timed as whole plans
    (graph replay, state resident): n = 20 complex128 U(2) + CZ layers
    (depth 10); n = 28 random pairs (depth 20) unfused and fused to
    k = 2..5 in complex64 and complex128; n = 32 random 1-3-qubit unitaries
    (depth 12) fused to k = 5 in complex64 and complex128; and at n = 32 the
    single-gate GB/s at every target plus k = 2, 3 gates on low, spread and
    high targets.  GB/s counts algorithmic bytes, TFLOP/s algorithmic flops."""
    cases = [("n20_u2cz_depth10", W.random_u2_cz(n=20, depth=10, seed=1000), None, ["c128"], [1, 5])]
    c2, p2 = W.random_u2_pairs(n=28, depth=20, seed=1001)
    cases.append(("n28_pairs_depth20", c2, p2, ["c64", "c128"], [1, 2, 3, 4, 5]))
    cases.append(("n32_dense123_depth12", W.random_dense_123(n=32, depth=12, seed=1002), None,
                  ["c64", "c128"], [5]))
    out = {}
    # per-gate GB/s by target position at n = 32: k = 1 at every target, and
    # k = 2, 3 Haar gates on low, spread and high target sets
    rng = np.random.default_rng(1006)
    sets = [(0, 1), (0, 31), (30, 31), (0, 1, 2), (0, 16, 31), (29, 30, 31)]
    for dt, S in (("c64", 8), ("c128", 16)):
        psi = torch.empty(1 << 32, dtype=torch.complex64 if dt == "c64" else torch.complex128,
                          device=dev)
        qsv.qsv_init_random(psi, 9)
        row = []
        for t in range(32):
            G = W.haar_unitary(rng, 2)
            tt = event_time(lambda: qsv.qsv_apply_gate(psi, (t,), (), G), 3, stream)
            row.append(round(2.0 * S * (1 << 32) / tt / 1e9, 1))
        multi = {}
        for ts in sets:
            G = W.haar_unitary(rng, 1 << len(ts))
            tt = event_time(lambda: qsv.qsv_apply_gate(psi, ts, (), G), 3, stream)
            multi[",".join(map(str, ts))] = round(2.0 * S * (1 << 32) / tt / 1e9, 1)
        out["n32_per_target_gbs_%s" % dt] = row
        out["n32_k23_gbs_%s" % dt] = multi
        del psi
        torch.cuda.empty_cache()
    for name, circ, params, dts, fuses in cases:
        for dt in dts:
            tdt = torch.complex64 if dt == "c64" else torch.complex128
            psi = torch.empty(1 << circ.n, dtype=tdt, device=dev)
            qsv.qsv_init_random(psi, 7)
            for k in fuses:
                plan = qsv.Plan(circ, qsv.C64 if dt == "c64" else qsv.C128, k, params_host=params)
                nl, b, f = plan.info()
                plan.run(psi)
                t = event_time(lambda: plan.run(psi), 3, stream)
                out["%s_%s_fuse%d" % (name, dt, k)] = {
                    "ms": round(t * 1e3, 3), "launches": nl, "gbs": round(b / t / 1e9, 1),
                    "hbm_frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4), "tflops": round(f / t / 1e12, 2)}
                del plan
            del psi
            torch.cuda.empty_cache()
    return out


def batched_leg(qsv, W, torch, np, dev):
    """1024 ansatz instances, n ~ U{12..22}, L ~ U{2..10}, complex64: energies
    and adjoint gradients of all instances per launch (autotuned once)."""
    insts = W.batched_hea()
    plan = qsv.BatchPlan(insts, qsv.C64, device=dev)
    params = torch.from_numpy(np.concatenate([i.params for i in insts])).to(dev)
    e = torch.empty(plan.ninst, dtype=torch.float64, device=dev)
    g = torch.empty(int(plan.offsets[-1]), dtype=torch.float64, device=dev)
    shape = plan.tune(params, e, g)
    plan.run(params, e, g)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run(params, e, g)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    unfused = 0.0
    for i in insts:
        N = float(1 << i.circuit.n)
        unfused += 6.0 * len(i.circuit.ops) * N * 8
    return {"workload": "1024 HEA instances, n~U{12..22}, L~U{2..10}, TFIM, complex64",
            "instance_grads_per_s": round(plan.ninst / t, 1), "ms_per_batch": round(t * 1e3, 2),
            "tuned_tile_qubits_threads_split": list(shape),
            "unfused_hbm_reference_ms": round(unfused / HBM_PEAK_GBS / 1e6, 1)}


def adjoint_leg(qsv, W, torch, np, dev):
    n, L = 20, 8
    circ, H = W.hea(n, L), W.tfim_chain(n)
    p = torch.from_numpy(W.random_params(circ.nparams, 1003)).to(dev)
    res = {"workload": "HEA n=20 L=8, TFIM", "nparams": circ.nparams}
    for name, code in [("c64", qsv.C64), ("c128", qsv.C128)]:
        plan = qsv.AdjointPlan(circ, H, code, 5, device=dev)
        e, g = plan.run(p)
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.run(p, e, g)
        torch.cuda.synchronize()
        ta = (time.perf_counter() - t0) / reps
        res[name + "_grads_per_s"] = round(1.0 / ta, 2)
        if name == "c64":
            # plain parameter shift on the same GPU: 2P energies, same forward plan
            pe = p.clone()
            en = torch.empty(1, dtype=torch.float64, device=dev)
            plan.energy(pe, en)
            vals = torch.empty(2 * circ.nparams, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for j in range(circ.nparams):
                for s, sign in enumerate((1.0, -1.0)):
                    pe.copy_(p)
                    pe[j] += sign * np.pi / 2
                    plan.energy(pe, en)
                    vals[2 * j + s].copy_(en[0])
            torch.cuda.synchronize()
            tps = time.perf_counter() - t0
            gps = 0.5 * (vals[0::2] - vals[1::2])
            res["param_shift_grads_per_s"] = round(1.0 / tps, 3)
            res["adjoint_over_param_shift"] = round(tps / ta, 1)
            res["max_abs_adjoint_minus_shift"] = float((gps - g).abs().max().cpu())
    return res


def adjoint_leg_large(qsv, W, torch, np, dev, n=26, L=8, nsub=8):
    """HEA at n = 26, L = 8 (416 parameters): full adjoint gradients/s in
    complex64 and complex128; plain parameter shift timed on a seeded subset
    of nsub parameters (2 nsub energies) and extrapolated to all of them;
    complex128 central finite differences (h = 1e-6) on the same subset as
    the accuracy check."""
    circ, H = W.hea(n, L), W.tfim_chain(n)
    P = circ.nparams
    p = torch.from_numpy(W.random_params(P, 1003)).to(dev)
    sub = np.sort(np.random.default_rng(26).choice(P, size=nsub, replace=False))
    res = {"workload": "HEA n=%d L=%d, TFIM" % (n, L), "nparams": P, "subset": [int(j) for j in sub]}
    for name, code in [("c64", qsv.C64), ("c128", qsv.C128)]:
        plan = qsv.AdjointPlan(circ, H, code, 5, device=dev)
        e, g = plan.run(p)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.run(p, e, g)
        torch.cuda.synchronize()
        ta = (time.perf_counter() - t0) / reps
        res[name + "_grads_per_s"] = round(1.0 / ta, 3)
        res[name + "_ms_per_gradient"] = round(ta * 1e3, 2)
        pe = p.clone()
        en = torch.empty(1, dtype=torch.float64, device=dev)
        plan.energy(pe, en)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        shift = []
        for j in sub:
            vals = []
            for sign in (1.0, -1.0):
                pe.copy_(p)
                pe[int(j)] += sign * np.pi / 2
                plan.energy(pe, en)
                vals.append(float(en.cpu()[0]))
            shift.append(0.5 * (vals[0] - vals[1]))
        tsub = time.perf_counter() - t0
        gsub = g.cpu().numpy()[sub]
        res[name + "_param_shift_grads_per_s_extrapolated"] = round(nsub / (tsub * P), 4)
        res[name + "_adjoint_over_param_shift"] = round(tsub * P / nsub / ta, 1)
        res[name + "_max_abs_adjoint_minus_shift"] = float(np.max(np.abs(np.array(shift) - gsub)))
        if name == "c128":
            h = 1e-6
            fd = []
            for j in sub:
                vals = []
                for sign in (1.0, -1.0):
                    pe.copy_(p)
                    pe[int(j)] += sign * h
                    plan.energy(pe, en)
                    vals.append(float(en.cpu()[0]))
                fd.append((vals[0] - vals[1]) / (2 * h))
            res["c128_max_abs_adjoint_minus_fd"] = float(np.max(np.abs(np.array(fd) - gsub)))
        del plan
        torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
