"""Benchmark of the MI355X variational-circuit hot path.

Headline workload: the 28-qubit random circuit on a 4x7 grid (20 cycles of
sqrt(X)/sqrt(Y)/sqrt(W) on every qubit plus fSim on one coupler pattern,
785 gates, complex128 state of 4 GiB resident in HBM).  One step = reset to
|0..0>, apply the whole circuit as fused HBM passes, read the norm and 1000
seeded output amplitudes.  value = gate applications per second.

Also reported:
* roofline of the dominant kernel (the fused forward pass), with its
  average duration measured by HIP events on the launch stream and the
  algorithmic bytes of one pass (read + write of every amplitude, 32 B/amp);
* the 20-qubit batched VQE gradient workload (64 parameter sets, 1600
  parameters, transverse-field Ising energy): gradients/s batched versus
  the same library run item by item;
* the noisy gradient (brick-wall circuit with one-qubit depolarizing and
  amplitude damping after every rotation, two-qubit depolarizing after every
  CZ, 20 layers) at n = 12 in both forms: states before each op recomputed
  from checkpoints, and Alg. 2 with channel inverses (two states); at n = 8
  also the oracle's inverse form on the host; and the batch of 32 such
  circuits with n in {8, 10, 12} (forward + backward per batch, both forms);
* bitstring sampling from the 28-qubit output state (2^20 samples, the
  paper's random-circuit sampling use) and measure! of one qubit;
* single unfused ops on the same state (dense one-, two- and three-qubit
  matrices, CZ) as GB/s against their algorithmic bytes;
* the surrogate's pieces at their working shapes (16 qubits, 10 layers, 320
  parameters; network 320 -> 512 -> 512 -> 1, batch 512): labels (energy and
  gradient) per second from the batched simulator, training steps per second
  (forward, backward with the gradient-matching term, Adam), and the BF16
  MFMA matrix product in TFLOP/s against the dense BF16 peak, at the
  network's layer shape and at 4096^3;
  and the optimiser comparison: wall-clock to a stated energy gap from one
  theta_0 for plain exact-gradient Adam over a step-size sweep against the
  surrogate-assisted loop (its labels and training included);
* the 12-qubit brick-wall circuit (20 layers of Rx, Ry, Rz on every qubit and
  CZ on alternating neighbour pairs, final state and <Z_0>): time per run;
* the per-gate sweep: H, Rx and CNOT alone on states of 14 to 30 qubits, on
  the lowest and the highest qubit, as GB/s against algorithmic bytes;
* cpu_baseline: the plain C oracle on this host, timed on a bounded prefix of
  the same 28-qubit circuit with all host threads, and with one.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-vqe] [--no-noisy]
                       [--no-surrogate] [--no-sweep]
       python bench.py --copy-calibration   (only a plain device copy of known
                                              size, for scaling HBM counters)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense
HERE = os.path.dirname(os.path.abspath(__file__))
# measured HBM traffic of the fused pass (rocprofv3 FETCH_SIZE / WRITE_SIZE,
# scaled by the same counters on a plain copy); used only while the kernel
# sources still have the digest recorded with the counters
TRAFFIC_FILE = os.path.join(HERE, "profiles", "rqc28_fused_pass_traffic.txt")
KERNEL_SOURCES = ["paper_2406_19212_amd/csrc/pass_kernels.h", "paper_2406_19212_amd/csrc/vqc_internal.h",
                  "paper_2406_19212_amd/csrc/inst_lds.hip", "paper_2406_19212_amd/csrc/jit_pass.h",
                  "paper_2406_19212_amd/csrc/jit.cpp", "paper_2406_19212_amd/csrc/api.cpp",
                  "paper_2406_19212_amd/build.py"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-vqe", action="store_true")
    ap.add_argument("--no-noisy", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true")
    return ap.parse_args()


def kernel_digest():
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(HERE, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """Bytes per pass from the committed counter summary, or None when the
    summary is missing or was taken on other kernel sources."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("source_digest") != kernel_digest():
            return None
        return float(kv["bytes_per_pass"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration(torch):
    """A plain copy of a 4 GiB buffer (2^28 complex128): reads 4 GiB and writes
    4 GiB per launch; run under rocprofv3 --pmc to get the counter scale."""
    n = 1 << 28
    x = torch.zeros(n, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": True, "bytes_read_per_launch": 16 * n,
                      "bytes_written_per_launch": 16 * n, "launches": 3}), flush=True)


def cpu_baseline(ops, n, seconds):
    """The oracle as it stands, on a prefix of the circuit (one gate at a time
    until `seconds` of work), reported in the same unit; then the same with
    one thread for half that time."""
    import oracle

    def timed(threads, secs):
        oracle.set_threads(threads)
        st = oracle.initial_state(n)
        done, t0 = 0, time.perf_counter()
        while done < len(ops) and time.perf_counter() - t0 < secs:
            oracle.apply_op_inplace(st, n, ops[done])
            done += 1
        dt = time.perf_counter() - t0
        del st
        return done, dt, oracle.get_threads()
    ops = list(ops)
    done, dt, used = timed(len(os.sched_getaffinity(0)), seconds)
    d1, dt1, used1 = timed(1, seconds / 2)
    return {"value": done / dt, "unit": "gate-apps/s", "cores": used, "kind": "oracle",
            "sample": "first %d of %d gates of the same 28-qubit circuit, one full-state pass each, %.1f s"
                      % (done, len(ops), dt),
            "single_thread": {"value": d1 / dt1, "cores": used1,
                              "sample": "first %d gates of the same circuit, %.1f s" % (d1, dt1)}}


def vqe_batched(torch, steps):
    """20-qubit HEA (40 layers, 1600 params), TFIM energy and adjoint gradient
    for 64 parameter sets: batched launches vs the same library item by item."""
    from paper_2406_19212_amd import Batch, Circuit, State
    from paper_2406_19212_amd import workloads as W
    n, L, Bn = 20, 40, 64
    ops = W.hea(n, L)
    P = W.count_params(ops)
    theta = torch.tensor(W.theta_uniform(W.CONFIG_SEED[2], Bn, P), device="cuda")
    terms = W.tfim(n, 1.0)
    circ = Circuit(n, ops, n_params=P)
    out = {}
    # plain: one item at a time
    st = State(n)
    grads = torch.zeros(Bn, P, dtype=torch.float64, device="cuda")

    def plain(k):
        for b in range(k):
            st.reset()
            circ.apply(st, theta[b])
            circ.backward(theta[b], st, terms, grad=grads[b], energy=False)
    plain(2)
    torch.cuda.synchronize()
    nb = 8
    t0 = time.perf_counter()
    plain(nb)
    torch.cuda.synchronize()
    out["plain_grads_per_s"] = nb / (time.perf_counter() - t0)
    try:
        states = [torch.empty(1 << n, dtype=torch.complex128, device="cuda") for _ in range(Bn)]
        bt = Batch([circ] * Bn, states, [theta[b] for b in range(Bn)])
        energies = torch.zeros(Bn, dtype=torch.float64, device="cuda")
        bgrads = [torch.zeros(P, dtype=torch.float64, device="cuda") for _ in range(Bn)]
        bt.capture(terms, bgrads, energies)
        bt.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            bt.replay()
        torch.cuda.synchronize()
        out["batched_grads_per_s"] = Bn * steps / (time.perf_counter() - t0)
        out["speedup_vs_plain"] = out["batched_grads_per_s"] / out["plain_grads_per_s"]
        # algorithmic bytes of one replay, per item: |0..0> written (16 B/amp),
        # forward passes (read + write, 32 B/amp), the energy with the seed
        # H|psi> (read psi, write Phi: 32 B/amp), adjoint passes over Phi and
        # Psi (64 B/amp); the gradient reduction's partials are negligible
        cs = circ.stats()
        nf, na = cs["n_passes"], cs["n_adj_passes"]
        per_item = float(1 << n) * (16 + 32 * nf + 32 + 64 * na)
        replay_s = Bn / out["batched_grads_per_s"]
        ach = Bn * per_item / replay_s / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(ach / HBM_PEAK_GBS, 4), "forward_passes": nf, "adjoint_passes": na,
                           "alg_bytes_per_replay": Bn * per_item, "replay_ms": round(1e3 * replay_s, 3),
                           "specialised": bool(cs["n_jit_passes"] and cs["n_jit_adj_passes"]),
                           "scope": "whole replay (every kernel) against its algorithmic bytes"}
    except Exception as e:  # report, do not hide
        out["batched_error"] = str(e)
    out.update({"workload": "hea-20q-40layers-1600params-tfim-batch64", "unit": "grads/s"})
    return out


def surrogate_leg(torch):
    """The surrogate's kernels at their working shapes: simulator labels,
    network training steps and the BF16 MFMA matrix product."""
    from paper_2406_19212_amd import surrogate as S
    from paper_2406_19212_amd.mlp import MLP, gemm_bf16
    out = {"workload": "hea-16q-10layers-320params-tfim; mlp-320-512-512-1-batch512"}
    sim = S.Simulator(16, 10, batch=256)
    count = 4096
    S.generate(sim, 256, 1)  # warm-up replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, E, G = S.generate(sim, count, 2)
    torch.cuda.synchronize()
    out["labels_per_s"] = round(count / (time.perf_counter() - t0), 1)
    del sim
    net = MLP(320, 512, 512, 512)
    S.init_params(net, 3)
    mu, sd = float(E.mean()), float(E.std())
    x = theta.float().contiguous()
    e = ((E - mu) / sd).float().contiguous()
    g = (G / sd).float().contiguous()
    nb = count // 512

    def train_steps(k):
        for i in range(k):
            s = (i % nb) * 512
            net.backward(x[s:s + 512], e[s:s + 512], g[s:s + 512], 1.0)
            net.adam(1e-3)
    train_steps(4)
    torch.cuda.synchronize()
    steps = 64
    t0 = time.perf_counter()
    train_steps(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["train_ms_per_step"] = round(1e3 * dt / steps, 4)
    out["train_samples_per_s"] = round(512 * steps / dt, 1)
    gem = {}
    for name, (M, N, K) in (("layer2_512x512x512", (512, 512, 512)), ("square_4096", (4096, 4096, 4096))):
        gen = torch.Generator(device="cpu").manual_seed(M + K)
        A = torch.randn(M, K, generator=gen).cuda()
        Bm = torch.randn(K, N, generator=gen).cuda()
        C = torch.zeros(M, N, dtype=torch.float32, device="cuda")
        reps = 20 if M < 4096 else 5
        gemm_bf16(A, Bm, C=C)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            gemm_bf16(A, Bm, C=C)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        tf = 2.0 * M * N * K / (ms * 1e-3) / 1e12
        gem[name] = {"ms": round(ms, 4), "TFLOP_per_s": round(tf, 2), "frac": round(tf / BF16_MFMA_PEAK_TFLOPS, 4)}
    out["gemm_bf16"] = gem
    out["gemm_peak_TFLOP_per_s"] = BF16_MFMA_PEAK_TFLOPS
    del net, theta, E, G, x, e, g
    torch.cuda.empty_cache()
    out["optimiser"] = S.compare()
    return out


def config0(torch, steps):
    """The 12-qubit brick-wall circuit: 20 layers of Rx, Ry, Rz on every qubit
    then CZ on alternating neighbour pairs; one run = reset, the circuit, the
    final state left in HBM and <Z_0> read back."""
    from paper_2406_19212_amd import Circuit, State
    from paper_2406_19212_amd import workloads as W
    n, L = 12, 20
    ops, theta = W.brickwall(n, L, W.CONFIG_SEED[0])
    circ = Circuit(n, ops, n_params=len(theta))
    th = torch.tensor(theta, dtype=torch.float64, device="cuda")
    st = State(n)
    z0 = [W.pauli_string({0: "z"}, 1.0)]

    def run():
        st.reset()
        circ.apply(st, th)
        return st.expectation(z0).real
    for _ in range(3):
        run()
    torch.cuda.synchronize()
    reps = max(50, 10 * steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        z = run()
    dt = time.perf_counter() - t0
    return {"workload": "brickwall-12q-20layers-rxryrz-cz", "gates": len(ops), "passes": circ.stats()["n_passes"],
            "ms_per_run": round(1e3 * dt / reps, 4), "gate_apps_per_s": round(len(ops) * reps / dt, 1),
            "z0": z, "runs": reps}


def gate_sweep(torch):
    """H, Rx(0.3) and CNOT applied alone (one kernel launch each) to states
    of 14 to 30 qubits, on the lowest qubit (CNOT: control 0, target 1) and
    on the highest (control n-2, target n-1): HIP events around repeated
    launches.  Algorithmic bytes: H and Rx read and write every amplitude (32
    B/amp); CNOT reads and writes only the control = 1 half (16 B/amp)."""
    from paper_2406_19212_amd import State
    from paper_2406_19212_amd.workloads import Op
    rows = []
    for n in range(14, 31):
        st = State(n)
        N = 1 << n
        reps = 50 if n < 24 else (10 if n < 29 else 4)
        for name, mk, bpa in (("h", lambda q: Op("h", (q,)), 32.0), ("rx", lambda q: Op("rx", (q,), (0.3,)), 32.0),
                              ("cnot", lambda q: Op("cnot", (q, q + 1)), 16.0)):
            for where, q in (("low", 0), ("high", n - 1 if name != "cnot" else n - 2)):
                op = mk(q)
                st.apply_op(op)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    st.apply_op(op)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                rows.append([n, name, where, round(ms * 1e3, 2), round(bpa * N / (ms * 1e-3) / 1e9, 1)])
        del st
        torch.cuda.empty_cache()
    return {"columns": ["n", "gate", "qubit", "us", "GB_per_s"], "rows": rows,
            "alg_bytes_per_amp": {"h": 32, "rx": 32, "cnot": 16}}


def single_ops(torch, st, n):
    """One unfused op per HBM pass on the 28-qubit state (Eqs. (3) and
    (twoqubitgate), Alg. 1 for three qubits): GB/s from HIP events on the
    launch stream, against the algorithmic bytes of each op kind."""
    from paper_2406_19212_amd import workloads as W
    from paper_2406_19212_amd.workloads import Op
    N = 1 << n
    cases = [("dense_1q_q27", Op("matrix", (27,), (), (), W.random_unitary(2, 1)), 32.0),
             ("dense_2q_q3_q27", Op("matrix", (3, 27), (), (), W.random_unitary(4, 2)), 32.0),
             ("dense_3q_q0_q13_q27", Op("matrix", (0, 13, 27), (), (), W.random_unitary(8, 3)), 32.0),
             ("cz_q5_q26", Op("cz", (5, 26)), 8.0)]
    out = {}
    for name, op, bpa in cases:
        st.apply_op(op)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            st.apply_op(op)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": round(ms, 4), "GB_per_s": round(bpa * N / (ms * 1e-3) / 1e9, 1),
                     "alg_bytes_per_amp": bpa}
    return out


def sampling(torch, st, n):
    """2^20 bitstrings from the 28-qubit output state (uniform numbers drawn
    on the host beforehand; host transfers of u and of the samples included),
    then measure! of qubit 0 with its collapse."""
    K = 1 << 20
    u = np.random.default_rng(7).uniform(size=K)
    st.sample(u[:1024])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = st.sample(u)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    o, p = st.measure(0, 0.5)
    torch.cuda.synchronize()
    dm = time.perf_counter() - t0
    return {"samples": K, "ms": round(1e3 * dt, 3), "samples_per_s": round(K / dt, 1),
            "distinct": int(np.unique(x).size), "measure_ms": round(1e3 * dm, 3),
            "measure_outcome": o, "measure_prob": p}


def noisy_backward(torch, with_cpu):
    """Noisy brick-wall gradient (20 layers, <Z0 Z1>): checkpointed versus
    inverse form on the GPU at n = 12, and at n = 8 beside the oracle."""
    from paper_2406_19212_amd import Circuit, State
    from paper_2406_19212_amd import workloads as W
    out = {"workload": "noisy-brickwall-20layers-zz01", "unit": "ms per gradient"}
    terms = W.zz(0, 1)
    for n in (12, 8):
        ops, th = W.noisy_brickwall(n, 20, W.CONFIG_SEED[3] + n)
        c = Circuit(n, ops, mixed=True, n_params=len(th))
        tht = torch.tensor(th, device="cuda")
        st = State(n, mixed=True)
        rec = {"ops": len(ops), "params": len(th), "passes": c.stats()["n_passes"]}
        res = {}
        for form in ("checkpoint", "inverse"):
            best = None
            for _ in range(3):
                st.reset()
                c.apply(st, tht)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if form == "checkpoint":
                    g, _ = c.backward(tht, st, terms, energy=False)
                else:
                    g, _ = c.backward_inverse(tht, st, terms, energy=False)
                torch.cuda.synchronize()
                dt = 1e3 * (time.perf_counter() - t0)
                best = dt if best is None else min(best, dt)
            rec[form + "_ms"] = round(best, 3)
            res[form] = g.cpu().numpy().copy()
        rec["max_grad_diff"] = float(np.max(np.abs(res["checkpoint"] - res["inverse"])))
        if n == 8 and with_cpu:
            import oracle
            t0 = time.perf_counter()
            _, g_ref, _ = oracle.grad_mixed_inverse(n, ops, th, terms)
            rec["oracle_inverse_ms"] = round(1e3 * (time.perf_counter() - t0), 1)
            rec["oracle_threads"] = oracle.get_threads()
            rec["max_diff_vs_oracle"] = float(np.max(np.abs(res["inverse"] - g_ref)))
        out["n%d" % n] = rec
        del st, c
    # 32 circuits of n in {8, 10, 12} per batch: forward + backward, both forms
    from paper_2406_19212_amd import Batch
    items = W.noisy_batch(W.CONFIG_SEED[3], 32, (8, 10, 12), 20)
    circs = [Circuit(n, ops, mixed=True, n_params=len(th)) for n, ops, th in items]
    states = [torch.empty(1 << (2 * n), dtype=torch.complex128, device="cuda") for n, *_ in items]
    thetas = [torch.tensor(th, device="cuda") for *_, th in items]
    grads = {f: [torch.zeros(t.numel(), dtype=torch.float64, device="cuda") for t in thetas]
             for f in ("checkpoint", "inverse")}
    en = torch.zeros(len(items), dtype=torch.float64, device="cuda")
    bt = Batch(circs, states, thetas)
    rec = {"circuits": len(items), "widths": [8, 10, 12]}
    for form in ("checkpoint", "inverse"):
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bt.forward()
            if form == "checkpoint":
                bt.backward(terms, grads[form], en)
            else:
                bt.backward_inverse(terms, grads[form], en)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        rec[form + "_s"] = round(best, 4)
        rec[form + "_circuits_per_s"] = round(len(items) / best, 2)
    rec["max_grad_diff"] = float(max((a - b).abs().max() for a, b in zip(grads["checkpoint"], grads["inverse"])))
    out["batch32"] = rec
    del bt, states
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    from paper_2406_19212_amd import Circuit, State
    from paper_2406_19212_amd import workloads as W

    n, rows, cols, cycles = 28, 4, 7, 20
    seed = W.CONFIG_SEED[1]
    ops = W.rqc_grid(rows, cols, cycles, seed)
    idx = W.rqc_bitstrings(n, 1000, seed + 1)
    t0 = time.perf_counter()
    circ = Circuit(n, ops)  # plans the fused passes and compiles them for this circuit
    create_s = time.perf_counter() - t0
    stats = circ.stats()
    st = State(n)

    def step():
        st.reset()
        circ.apply(st)
        nrm = st.norm()
        amps = st.gather(idx)
        return nrm, amps

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nrm, amps = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    gate_apps = len(ops) * args.steps / dt

    # roofline: per-pass durations from HIP events on the launch stream
    st.reset()
    pass_ms = circ.apply_timed(st)
    amps_n = 1 << n
    pass_bytes = 32.0 * amps_n  # algorithmic: read + write every amplitude once per pass
    avg_ms = float(np.mean(pass_ms))
    achieved = pass_bytes / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": ("vqc_jf0..%d (k_pass_lds<%d,%d,0> driver specialised per pass)"
                       % (stats["n_passes"] - 1, stats["tile_bits"], stats["reg_bits"])
                       if stats["n_jit_passes"] else "k_pass_lds<%d,%d,0>" % (stats["tile_bits"], stats["reg_bits"])),
            "avg_pass_ms": round(avg_ms, 4), "passes": stats["n_passes"], "bytes_per_pass": pass_bytes,
            "kernel_digest": kernel_digest()}

    rec = {"metric": "28q gate-apps/s", "value": round(gate_apps, 1), "unit": "gate-apps/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "rqc-4x7-28q-20cycles", "n_qubits": n, "gates": len(ops),
                      "fsim": sum(1 for o in ops if o.name == "fsim"), "seed": seed,
                      "passes": stats["n_passes"], "tile_bits": stats["tile_bits"],
                      "low_bits": stats["low_bits"], "reg_bits": stats["reg_bits"],
                      "specialised_passes": stats["n_jit_passes"], "compile_s": round(stats["jit_ms"] / 1e3, 2),
                      "code_cached": stats["jit_cached"], "circuit_create_s": round(create_s, 2),
                      "norm_minus_1": float(nrm - 1.0),
                      "mean_2n_abs2": float(np.mean(np.abs(amps) ** 2) * amps_n)},
           "roofline": roof}
    rec["sampling"] = sampling(torch, st, n)
    rec["single_ops"] = single_ops(torch, st, n)
    del st
    torch.cuda.empty_cache()
    if not args.no_vqe:
        rec["vqe_batched"] = vqe_batched(torch, max(1, args.steps // 5))
        torch.cuda.empty_cache()
    if not args.no_noisy:
        rec["noisy_backward"] = noisy_backward(torch, not args.no_cpu)
        torch.cuda.empty_cache()
    if not args.no_surrogate:
        rec["surrogate"] = surrogate_leg(torch)
        torch.cuda.empty_cache()
    rec["brickwall12"] = config0(torch, args.steps)
    if not args.no_sweep:
        rec["gate_sweep"] = gate_sweep(torch)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(ops, n, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
