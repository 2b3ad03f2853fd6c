#!/usr/bin/env python3
"""Benchmark of the local-energy path on one MI355X.

One step = one pass of the hot path over one batch already resident in HBM:
E_loc (Eq. 5: the pair join's grouping and pair kernel, or the sample hash
and the enumeration / streaming lookups, then the finish kernel) and the
weighted energy and variance over it (Eq. 1), one nqs_eloc_energy call, which
synchronises.  The
Pauli table is built and uploaded once before the timed region (it is
resident across VMC steps); its setup time is reported separately.

Default workload: 100 qubits (50 orbitals, 25 alpha + 25 beta, integral
decay length 6), full Jordan-Wigner table (1,963,674 X groups, 9,256,243
terms), 262,144 unique sector samples with geometric counts, log|psi| ~
N(0, 2), phase ~ U[0, 2 pi), FP64; the FP32-with-compensation form is timed
beside it.  Secondary lines: the 40-qubit batch (65,536 samples) and the
latency of the 12-qubit batch (400 samples) in microseconds.

Prints ONE JSON line.  Metric: E_loc pair-evaluations per second, where a
pair is one (unique sample, X group) combination, N_s * G per batch.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: int32 VALU lane-operations per second
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# FP64 adds per second: one v_add_f64 per lane per clock (78.6 TFLOP/s counts
# an FMA as two)
FP64_PEAK_ADDS = 256 * 4 * 16 * 2.4e9
CSRC = os.path.join(ROOT, "paper_2506_23809_amd", "csrc")
# int8 dense MFMA peak of MI355X (5.0 POP/s)
INT8_PEAK_OPS = 5.0e15
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash(kernel: str) -> str:
    """Hash of the source file that defines the kernel."""
    src = "nqs_join.hip" if kernel.startswith("join_") else "nqs_kernels.hip"
    with open(os.path.join(CSRC, src), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_bytes(n_s, words, n_groups, n_terms, probes, hits, hit_terms):
    """Bytes the method must move for one batch: samples in (key, a, phi),
    E_loc out, one 32-byte granule per lookup, the table once, and for each
    hit the partner's (a, phi) plus the hit group's terms."""
    wb = 8 * words
    return (n_s * (wb + 24 + 16) + probes * 32 + (n_groups + n_terms) * (wb + 8)
            + hits * 16 + hit_terms * (wb + 8))


def algorithmic_ops_per_sample_diag(n_qubits):
    """Integer work of the exact occupation-form diagonal per sample on the
    int8 matrix cores: a multiply-add (two operations) of each of the 8
    digits of each of the n_qubits (n_qubits + 1) / 2 terms of the triangle."""
    return 2 * 8 * n_qubits * (n_qubits + 1) // 2


def algorithmic_bytes_join_pairs(entries, candidates):
    """Bytes the pair kernel's launch moves in the naive per-entry model: per
    entry (sample, block) its packed entry and group range (16 B), its bit
    string (16 B) and its partial sum out (16 B); per candidate (another
    member of its group) the partner's entry (8 B) and bit string (16 B).
    (The timed launches only join: the grouping made the sample checks, and
    no hash build rides along.)"""
    return 48 * entries + 24 * candidates


def algorithmic_ops_per_probe_enum():
    """Integer work of the flip enumeration per probe (one spin-conserving
    flip of one sample): one XOR forming h(x ^ X) from the row and column
    hashes, the filter word offset (shift, mask), the two filter bits (a
    shift by h, a shift of h, a shift by that) and their AND, and the shift-OR
    that records the outcome in the lane's row mask."""
    return 1 + 2 + 4 + 1


def algorithmic_ops_per_candidate_join(words):
    """Integer work of the pair join per candidate (an ordered pair of samples
    sharing a group: one bucket and content fingerprint): the XOR of the two
    bit strings and its popcount (one 32-bit operation per half word each),
    and the compare against the largest flip."""
    return 2 * words + 2 * words + 1


def algorithmic_ops_per_entry_join(words):
    """Integer work of the join's grouping per entry (sample, block): the
    block's hash (one XOR per occupied qubit, about a fifth of 2 * 32 * words
    bits set) and its bucket (multiply, shift), the count, the scatter and
    the place in its sorted bucket (one atomic and a few moves each)."""
    return (2 * 32 * words) // 10 + 2 + 6


def algorithmic_ops_per_pair(n_qubits, spin_bits):
    """Integer work the method needs per (sample, group) pair: the exact
    sector test on the alpha and beta fields (AND + POPC each, one
    combine and one compare) and one XOR forming the hash of x ^ X.  Fields
    of up to 32 bits take one 32-bit operation, up to 64 bits two."""
    words = 1 if spin_bits <= 32 else 2
    return 2 * (2 * words) + 2 + 1


def cpu_baseline(w, threads, e_loc_gpu=None, energies=None, budget_s=20.0):
    """The oracle as it stands, on the host cores, on a bounded sample.  When
    the whole batch fits in the budget, the oracle's local energies and Eq. 1
    energy are also set beside the GPU's (e_loc_gpu: FP64 E_loc; energies:
    (FP64, FP32-compensated) mean energies)."""
    import numpy as np
    import oracle
    n = w.n_samples
    G = oracle.n_groups(w.x)
    rows = np.arange(min(n, 256), dtype=np.int64)
    t0 = time.perf_counter()
    oracle.eloc_rows(w.n_qubits, w.x, w.z, w.c, w.samples, w.log_amp, w.phase, rows,
                     threads=threads)
    t_probe = time.perf_counter() - t0
    per_row = t_probe / len(rows)
    check = None
    if per_row * n <= budget_s:
        t0 = time.perf_counter()
        ref, ab, _ = oracle.eloc(w.n_qubits, w.x, w.z, w.c, w.samples, w.log_amp, w.phase,
                                 threads=threads)
        dt = time.perf_counter() - t0
        done = n
        sample = f"all {n} samples (full S x S double loop)"
        m_ref, _, _ = oracle.energy(w.weights, ref)
        check = {"energy_re_oracle": m_ref.real}
        if e_loc_gpu is not None:
            check["max_err_eloc_fp64_rel_to_abs_sum"] = float(np.max(np.abs(e_loc_gpu - ref) / ab))
        if energies is not None:
            check["abs_err_re_energy_fp64_Ha"] = abs(energies[0].real - m_ref.real)
            check["abs_err_re_energy_fp32k_Ha"] = abs(energies[1].real - m_ref.real)
    else:
        m = max(256, int(budget_s / per_row))
        sel = np.random.default_rng(0).choice(n, size=m, replace=False).astype(np.int64)
        t0 = time.perf_counter()
        oracle.eloc_rows(w.n_qubits, w.x, w.z, w.c, w.samples, w.log_amp, w.phase, sel,
                         threads=threads)
        dt = time.perf_counter() - t0
        done = m
        sample = f"{m} of {n} sample rows, each against all {n} samples"
    res = {"value": done * G / dt, "unit": "pair-evals/s", "cores": threads,
           "kind": "oracle", "sample": sample, "seconds": round(dt, 3),
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if check is not None:
        res["check"] = check
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="nq100", choices=["nq12", "nq40", "nq100"])
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 40-qubit and 12-qubit secondary measurements")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32k"])
    ap.add_argument("--filter-bits", type=int, default=0,
                    help="on-chip filter bits per sample (0: the library's default)")
    ap.add_argument("--strategy", default="auto", choices=["auto", "stream", "enum", "join"],
                    help="lookup strategy: group streaming, flip enumeration or pair join "
                         "(auto: the device picks by counted cost)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-strategy-compare", action="store_true",
                    help="skip the forced-enumeration comparison run (profiler passes)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--mode", default="single", choices=["single", "batched", "serve", "copy"],
                    help="single: the headline step; batched: 32 Hamiltonians in one "
                         "persistent graph-captured launch; serve: continuous batching loop; "
                         "copy: a plain 1 GiB device copy, the calibration of the HBM byte "
                         "counters")
    ap.add_argument("--jobs", type=int, default=32, help="Hamiltonians in the batched family")
    ap.add_argument("--requests", type=int, default=2000,
                    help="serve: requests per point of the sweep")
    ap.add_argument("--rates", default="200,1000,2000,3000,4000,inf",
                    help="serve: aggregate arrival rates per second to sweep (inf: all at once)")
    ap.add_argument("--tuning-cache", default=os.path.join(ROOT, "paper_2506_23809_amd",
                                                           "tuning_mi355x.json"))
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              f"the sharded path is not run.", file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2506_23809_amd as nqs
    import workloads

    def log(msg):
        if not args.quiet:
            print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.mode == "batched":
        return run_batched(args, log)
    if args.mode == "serve":
        import serve_bench
        return serve_bench.run(args, log)
    if args.mode == "copy":
        return run_copy(args, log)

    t0 = time.perf_counter()
    w = workloads.workload(args.workload)
    log(f"workload {w.name}: {w.n_samples} samples, {w.x.shape[0]} terms "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    if args.strategy != "auto" or args.filter_bits:
        ham.set_tuning(filter_bits=args.filter_bits, strategy=args.strategy)
    G, T, table_bytes = ham.info()
    words = 1 if w.n_qubits <= 63 else 2
    log(f"table: {G} groups, {T} terms, {table_bytes / 1e6:.1f} MB, setup {setup_ms:.1f} ms")

    S = nqs.to_device_samples(w.samples, dev)
    la = torch.from_numpy(w.log_amp).to(dev)
    ph = torch.from_numpy(w.phase).to(dev)
    wt = torch.from_numpy(w.weights).to(dev)
    out = torch.empty((w.n_samples, 2), dtype=torch.float64, device=dev)

    def timed(precision):
        """Warm-up, then EXACTLY args.steps timed steps of one precision.

        The timed steps call nqs_eloc_energy (E_loc, then Eq. 1 over it,
        one launch sequence) with the same arguments each time, as a VMC loop
        does: after its first calls the library replays the step as one
        captured HIP graph.  Then as many profiled steps (eager launches, HIP
        events around every stage on the launch stream) give the per-kernel
        durations and the eager step time."""
        def step():
            return ham.eloc_energy_into(out, S, la, ph, wt, precision=precision)

        for k in range(args.warmup):
            step()
            log(f"{precision} warmup {k + 1}/{args.warmup}")
        ham.sync()
        st = ham.stats()
        per_step = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            mean, var, sw = step()          # nqs_eloc_energy synchronises the stream
            per_step.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ham.sync()
        ms = elapsed * 1e3 / args.steps
        # profiled steps: eager, every stage timed
        ham.profile(True)
        kms, per_eager = [], []
        torch.cuda.synchronize()
        for k in range(args.steps):
            ts = time.perf_counter()
            step()
            per_eager.append((time.perf_counter() - ts) * 1e3)
            kms.append(ham.last_stage_ms())
        torch.cuda.synchronize()
        ham.profile(False)
        ham.sync()
        log(f"{precision}: timed {args.steps} steps: {ms:.3f} ms/step (graph replay), "
            f"{np.mean(per_eager):.3f} ms/step eager and profiled, E = {mean.real:.10f}, "
            f"var = {var:.4e}")
        timed.per_step[precision] = per_step
        timed.eager[precision] = per_eager
        return ms, np.array(kms), mean, var, sw, st

    timed.per_step = {}
    timed.eager = {}
    other = "fp32k" if args.precision == "fp64" else "fp64"
    ms_per_step, kms, mean, var, sw, st = timed(args.precision)
    o_ms, o_kms, o_mean, o_var, _, _ = timed(other)
    e_fp64 = mean if args.precision == "fp64" else o_mean
    e_fp32k = o_mean if args.precision == "fp64" else mean
    e_loc_fp64 = None
    if args.precision == "fp64":
        ham.eloc_into(out, S, la, ph, wt, precision="fp64")
        ham.sync()
        e_loc_fp64 = torch.view_as_complex(out).cpu().numpy()

    kms = np.array(kms)
    group_ms, build_ms, pair_ms, lookup_ms, finish_ms, total_ms = (
        float(v) for v in kms.mean(axis=0))
    pairs = st["pairs"]
    value = pairs / (ms_per_step / 1e3)
    plan = ham.plan()
    joined = plan.get("join_ran") == 1
    enumerated = st.get("enum_rounds", 0) > 0
    strategy = "pair join" if joined else ("enumeration" if enumerated else "streaming")
    n_occ = w.n_alpha + w.n_beta
    occ_form = True  # every molecular table has the occupation-form diagonal
    finish_name = "eloc_finish_mfma_kernel" if occ_form else "eloc_finish_kernel"
    # the single kernels of the step and their live durations (HIP events
    # around each on the launch stream); the grouping stage is several
    # launches and is reported beside them
    if joined:
        kernels = {"join_pair_kernel": pair_ms, finish_name: finish_ms}
    elif enumerated:
        kernels = {"eloc_enum_kernel": lookup_ms, finish_name: finish_ms}
    else:
        kernels = {"eloc_lookup_kernel": lookup_ms, finish_name: finish_ms}
    kernel_name = max(kernels, key=kernels.get)
    kernel_ms = kernels[kernel_name]
    entries = plan["join_blocks"] * w.n_samples if joined else 0
    if kernel_name == finish_name:
        # exact occupation-form diagonal on the int8 matrix cores: per sample
        # the quadratic form over the nq (nq + 1) / 2 terms of the triangle,
        # each a multiply-add of 8 digits
        bound, unit = "mfma", "TOP/s (int8, dense)"
        peak = INT8_PEAK_OPS
        per_unit = algorithmic_ops_per_sample_diag(w.n_qubits)
        units = w.n_samples
        unit_name = "sample (int8 digit multiply-adds of the diagonal's triangle, x2)"
        achieved = per_unit * units / (kernel_ms / 1e3)
    elif kernel_name == "join_pair_kernel":
        bound, unit = "hbm", "GB/s"
        peak = HBM_PEAK_GBS * 1e9
        per_unit = None
        units = {"entries": entries, "candidates": st["candidates"]}
        unit_name = "entry (sample, block): 48 B; candidate pair inside a group: 24 B"
        b_pair = algorithmic_bytes_join_pairs(entries, st["candidates"])
        achieved = b_pair / (kernel_ms / 1e3)
    elif kernel_name == "eloc_enum_kernel":
        bound, unit = "alu", "Tops/s (int32 VALU lane-ops)"
        peak = VALU_PEAK_OPS
        per_unit = algorithmic_ops_per_probe_enum()
        units = st["probes"]
        unit_name = "probe"
        achieved = per_unit * units / (kernel_ms / 1e3)
    else:
        bound, unit = "alu", "Tops/s (int32 VALU lane-ops)"
        peak = VALU_PEAK_OPS
        per_unit = algorithmic_ops_per_pair(w.n_qubits, w.K)
        units = pairs
        unit_name = "pair"
        achieved = per_unit * units / (kernel_ms / 1e3)
    scale = 1e9 if bound == "hbm" else 1e12

    traffic = None
    # HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes of this
    # kernel and workload, valid only for the kernel source they were taken on
    traffic_file = os.path.join(PROFILES, f"traffic_{kernel_name}_{w.name}.json")
    if os.path.exists(traffic_file):
        try:
            with open(traffic_file) as f:
                tr = json.load(f)
            if tr.get("kernel_source_sha256_16") == kernel_source_hash(kernel_name) and \
                    tr.get("workload") == w.name and tr.get("kernel") == kernel_name:
                traffic = tr.get("hbm_bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    # the method's bytes for the whole batch as the SURVEY counts them (one
    # 32-byte granule per sector-passing lookup, the table once)
    n_diag_terms = int(np.sum((w.x[:, 0] == 0) & (w.x[:, 1] == 0)))
    hit_terms = st["terms"] - w.n_samples * n_diag_terms
    b_alg = algorithmic_bytes(w.n_samples, words, G, T, st["probes"], st["hits"], max(hit_terms, 0))

    res = {
        "metric": "E_loc pair-evals/s",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_median": float(np.median(timed.per_step[args.precision])),
        "ms_per_step_min": float(np.min(timed.per_step[args.precision])),
        "ms_per_step_eager_profiled": float(np.mean(timed.eager[args.precision])),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+kahan/f64",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {w.n_qubits} qubits ({w.K} orbitals, {w.n_alpha}a+{w.n_beta}b), "
                        f"{w.n_samples} unique sector samples, geometric counts, "
                        f"log|psi|~N(0,2), phase~U[0,2pi), JW table G={G} T={T}",
            "n_qubits": w.n_qubits, "n_samples": w.n_samples, "n_groups": G, "n_terms": T,
            "precision": args.precision,
        },
        "roofline": {
            "kernel": kernel_name,
            "bound": bound,
            "achieved": achieved / scale,
            "peak": peak / scale,
            "unit": unit,
            "frac": achieved / peak,
            "traffic": traffic,
            "traffic_GBps": (traffic / (kernel_ms / 1e3) / 1e9) if traffic else None,
            "algorithmic_per_unit": per_unit,
            "unit_of_work": unit_name,
            "units_per_launch": units,
            "kernel_ms": kernel_ms,
            "step_kernels_ms": {
                "hash_clear_and_join_grouping": group_ms, "hash_build": build_ms,
                "join_pair_kernel": pair_ms, "enum_or_stream_lookup": lookup_ms,
                finish_name: finish_ms, "evaluation_total": total_ms},
            "method_bytes": {
                "algorithmic_bytes_per_batch": b_alg,
                "GBps_over_step": b_alg / (ms_per_step / 1e3) / 1e9,
                "note": "one 32-byte granule per sector-passing lookup and the table once; "
                        "the pair join touches neither for unconnected samples",
            },
        },
        "strategy": strategy,
        "plan": plan,
        "kernel_ms": {"hash_clear_and_join_grouping": group_ms, "hash_build": build_ms,
                      "join_pairs": pair_ms, "lookup": lookup_ms, "finish": finish_ms},
        "counts": st,
        "probes_per_s": st["probes"] / (ms_per_step / 1e3),
        "setup_ms": setup_ms,
        "energy": {"re": mean.real, "im": mean.imag, "var": var, "sum_w": sw},
        "compare": {
            "precision": other,
            "value": pairs / (o_ms / 1e3),
            "ms_per_step": o_ms,
            "ms_per_step_median": float(np.median(timed.per_step[other])),
            "ms_per_step_min": float(np.min(timed.per_step[other])),
            "kernel_ms": dict(zip(("hash_clear_and_join_grouping", "hash_build", "join_pairs",
                                   "lookup", "finish", "evaluation_total"),
                                  (float(v) for v in np.array(o_kms).mean(axis=0)))),
            "energy_re": o_mean.real,
            "abs_err_re_energy_fp32k_vs_fp64_Ha": abs(e_fp32k.real - e_fp64.real),
        },
    }
    if joined and ham.plan().get("join_ran") == 1 and not args.no_strategy_compare:
        res["compare_strategy"] = compare_enumeration(ham, out, S, la, ph, wt, args, log, pairs)
    ham.close()
    if not args.no_secondary:
        res["secondary"] = secondary(args, log, dev)
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"cpu baseline: oracle on {threads} threads")
        res["cpu_baseline"] = cpu_baseline(w, threads, e_loc_fp64, (e_fp64, e_fp32k))
        log(f"cpu baseline: {res['cpu_baseline']}")
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


def compare_enumeration(ham, out, S, la, ph, wt, args, log, pairs):
    """The same FP64 step with the flip enumeration forced (the strategy the
    device declines here): its time and its kernel's VALU roofline."""
    import numpy as np

    import paper_2506_23809_amd as nqs
    ham.set_tuning(strategy="enum")
    for _ in range(args.warmup):
        ham.eloc_energy_into(out, S, la, ph, wt)
    ham.sync()
    ham.profile(True)
    per, kms = [], []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        ham.eloc_energy_into(out, S, la, ph, wt)
        per.append((time.perf_counter() - t0) * 1e3)
        kms.append(ham.last_kernel_ms())
    ham.profile(False)
    ham.sync()
    st = ham.stats()
    ham.set_tuning(strategy="auto")
    k_ms = float(np.mean([k[1] for k in kms]))
    achieved = algorithmic_ops_per_probe_enum() * st["probes"] / (k_ms / 1e3)
    ms = float(np.mean(per))
    log(f"enumeration forced: {ms:.3f} ms/step, kernel {k_ms:.3f} ms")
    return {"strategy": "enumeration", "ms_per_step": ms,
            "ms_per_step_median": float(np.median(per)), "ms_per_step_min": float(np.min(per)),
            "value": pairs / (ms / 1e3), "kernel": "eloc_enum_kernel", "kernel_ms": k_ms,
            "roofline_frac": achieved / VALU_PEAK_OPS, "achieved_Tops": achieved / 1e12,
            "probes": st["probes"], "hits": st["hits"]}


def secondary(args, log, dev):
    """The other single-GPU workloads, timed the same way (not the headline):
    the 40-qubit batch's throughput and the 12-qubit batch's latency."""
    import numpy as np
    import torch

    import paper_2506_23809_amd as nqs
    import workloads

    out = {}
    for name in ("nq40", "nq12"):
        if name == args.workload:
            continue
        w = workloads.workload(name)
        ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
        S = nqs.to_device_samples(w.samples, dev)
        la = torch.from_numpy(w.log_amp).to(dev)
        ph = torch.from_numpy(w.phase).to(dev)
        wt = torch.from_numpy(w.weights).to(dev)
        e = torch.empty((w.n_samples, 2), dtype=torch.float64, device=dev)
        steps = max(args.steps, 50) if name == "nq12" else args.steps
        for _ in range(args.warmup):
            ham.eloc_energy_into(e, S, la, ph, wt)
        ham.sync()
        per = []
        for _ in range(steps):
            t0 = time.perf_counter()
            ham.eloc_energy_into(e, S, la, ph, wt)
            per.append((time.perf_counter() - t0) * 1e3)
        ham.sync()
        st = ham.stats()
        pairs = st["pairs"]
        ms = float(np.mean(per))
        plan = ham.plan()
        strategy = ("pair join" if plan["join_ran"] == 1 else
                    ("enumeration" if st["enum_rounds"] > 0 else "streaming"))
        out[w.name] = {"pair_evals_per_s": pairs / (ms / 1e3), "ms_per_step": ms,
                       "ms_per_step_median": float(np.median(per)),
                       "ms_per_step_min": float(np.min(per)), "steps": steps,
                       "latency_us_median": float(np.median(per)) * 1e3,
                       "strategy": strategy, "counts": st}
        log(f"secondary {w.name}: {ms:.3f} ms/step (median {np.median(per):.3f})")
        ham.close()
    return out


def cpu_model() -> str:
    """The host CPU's model name (what lscpu prints), from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _family(n_jobs, log):
    import workloads
    t0 = time.perf_counter()
    fam = [workloads.batched_family(j) for j in range(n_jobs)]
    log(f"family of {n_jobs}: qubits {[w.n_qubits for w in fam]}, samples "
        f"{[w.n_samples for w in fam]} ({time.perf_counter() - t0:.1f} s to generate)")
    return fam


def run_copy(args, log):
    """A plain device copy of known size (1 GiB read, 1 GiB written per step):
    rocprofv3's FETCH_SIZE and WRITE_SIZE of this copy give the factor that
    turns the counters of the E_loc kernels into bytes."""
    import torch

    n_bytes = 1 << 30
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(json.dumps({"metric": "device copy GB/s", "value": 2 * n_bytes / (ms / 1e3) / 1e9,
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "copy of 1 GiB (read 1 GiB, write 1 GiB)",
                                 "bytes_read": n_bytes, "bytes_written": n_bytes}}), flush=True)


def run_batched(args, log):
    """Many Hamiltonians with uneven batches: serial single launches versus one
    batched persistent launch versus its captured HIP graph, FP64 and FP32."""
    import numpy as np
    import torch

    import paper_2506_23809_amd as nqs

    fam = _family(args.jobs, log)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream()
    hams, bufs = [], []
    for w in fam:
        hams.append(nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks))
        bufs.append((nqs.to_device_samples(w.samples, dev), torch.from_numpy(w.log_amp).to(dev),
                     torch.from_numpy(w.phase).to(dev), torch.from_numpy(w.weights).to(dev),
                     torch.empty((w.n_samples, 2), dtype=torch.float64, device=dev)))
    pairs = sum(h.n_groups * w.n_samples for h, w in zip(hams, fam))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tunings = []
    with torch.cuda.stream(stream):
        for h, (S, la, ph, wt, out) in zip(hams, bufs):
            tunings.append(h.autotune(S, la, ph, out, cache_path=args.tuning_cache)[0])
    stream.synchronize()
    log(f"autotune: {time.perf_counter() - t0:.1f} s ({len(hams)} jobs, cache {args.tuning_cache})")

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        stream.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        stream.synchronize()
        return (time.perf_counter() - t) * 1e3 / steps

    res = {}
    for prec in ("fp64", "fp32k"):
        def serial():
            for h, (S, la, ph, wt, out) in zip(hams, bufs):
                h.eloc_into(out, S, la, ph, wt, precision=prec, stream=stream)
        ms_serial = timed(serial, args.steps, args.warmup)
        batch = nqs.Batch([(h, *b) for h, b in zip(hams, bufs)], precision=prec, stream=stream)
        ms_batch = timed(lambda: batch.launch(stream), args.steps, args.warmup)
        batch.capture(stream)
        ms_graph = timed(lambda: batch.replay(stream), args.steps, args.warmup)
        for h in hams:
            h.sync(stream)
        batch.close()
        res[prec] = {"serial_ms": ms_serial, "batched_ms": ms_batch, "graph_ms": ms_graph,
                     "graph_pair_evals_per_s": pairs / (ms_graph / 1e3),
                     "serial_pair_evals_per_s": pairs / (ms_serial / 1e3)}
        log(f"{prec}: serial {ms_serial:.2f} ms, batched {ms_batch:.2f} ms, graph {ms_graph:.2f} ms")
    best = res["fp32k"]
    out = {
        "metric": "E_loc pair-evals/s (batched Hamiltonian family)",
        "value": best["graph_pair_evals_per_s"],
        "unit": "pair-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": best["graph_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+kahan/f64", "data": "synthetic",
        "config": {"workload": f"{len(fam)} Hamiltonians, qubits 24..80 at half filling, "
                               f"samples log-uniform in [1e3, 2e5], geometric counts",
                   "n_qubits": [w.n_qubits for w in fam], "n_samples": [w.n_samples for w in fam],
                   "pairs": pairs, "tunings": tunings},
        "by_precision": res,
        "speedup_graph_fp32k_vs_serial_fp64": res["fp64"]["serial_ms"] / best["graph_ms"],
    }
    for h in hams:
        h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
