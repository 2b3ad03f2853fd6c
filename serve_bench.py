"""Serving leg of bench.py: synthetic VMC jobs issuing E_loc requests.

64 jobs are drawn from the batched-family distribution (qubits 24..80 at
half filling, samples log-uniform in [1e3, 2e5]); each keeps its Hamiltonian
resident and alternates between two sample batches (with their psi values).
Requests arrive as a Poisson process (200 per second in aggregate by
default), each for a uniformly chosen job.  The same arrival trace is
replayed through three server configurations:

* serial FP64: one stream, one request per launch (plain FP64 launches in
  arrival order);
* continuous FP64 and continuous FP32+compensation: four streams, up to 64
  requests per launch, admission by HBM footprint (64 GB budget).

Reported: completed requests per second, pair-evaluations per second and
the p50 / p99 latency from submission to completion.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np

SEED = 4
HBM_BUDGET = 64 * 1024 ** 3


def make_jobs(n_jobs, log, max_qubits=None, max_samples=None):
    import workloads
    t0 = time.perf_counter()
    jobs = []
    for j in range(n_jobs):
        w = workloads.batched_family(j, seed=SEED)
        jobs.append(w)
    log(f"{n_jobs} serving jobs generated in {time.perf_counter() - t0:.1f} s")
    return jobs


def second_batch(w, j):
    """A second sample batch (and psi) for job j from its own seed prefix."""
    import workloads
    rng = np.random.default_rng([SEED, 100 + j, 11])
    s = workloads.sector_samples(rng, w.K, w.n_alpha, w.n_beta, w.n_samples)
    la = np.random.default_rng([SEED, 100 + j, 13]).normal(0.0, 2.0, w.n_samples)
    ph = np.random.default_rng([SEED, 100 + j, 14]).uniform(0.0, 2 * math.pi, w.n_samples)
    return s, la, ph


def poisson_trace(n_requests, rate, n_jobs):
    rng = np.random.default_rng([SEED, 99])
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    job = rng.integers(0, n_jobs, size=n_requests)
    return arrivals, job


def replay(server, hams, payloads, arrivals, job_of):
    """Submit the trace in real time; returns (latencies us, wall s)."""
    counter = [0] * len(hams)
    lat = {}
    t0 = time.perf_counter()
    for k, (t_arr, j) in enumerate(zip(arrivals, job_of)):
        delay = t0 + t_arr - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        p = payloads[j][counter[j] % 2]
        counter[j] += 1
        server.submit(hams[j], *p)
        for t, us in server.poll():
            lat[t] = us
    server.drain(600.0)
    wall = time.perf_counter() - t0
    for t, us in server.poll():
        lat[t] = us
    return np.array(sorted(lat.values())), wall


def run(args, log):
    import torch

    import paper_2506_23809_amd as nqs

    n_jobs = 64
    n_req = getattr(args, "requests", 0) or 400
    rate = getattr(args, "rate", 0.0) or 200.0
    jobs = make_jobs(n_jobs, log)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    hams, payloads, pairs = [], [], []
    for j, w in enumerate(jobs):
        h = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
        hams.append(h)
        s2, la2, ph2 = second_batch(w, j)
        p = []
        for s, la, ph in ((w.samples, w.log_amp, w.phase), (s2, la2, ph2)):
            p.append((nqs.to_device_samples(s, dev), torch.from_numpy(la).to(dev),
                      torch.from_numpy(ph).to(dev), torch.from_numpy(w.weights).to(dev),
                      torch.empty((w.n_samples, 2), dtype=torch.float64, device=dev)))
        payloads.append(p)
        pairs.append(h.n_groups * w.n_samples)
    torch.cuda.synchronize()
    arrivals, job_of = poisson_trace(n_req, rate, n_jobs)
    req_pairs = float(sum(pairs[j] for j in job_of))
    log(f"trace: {n_req} requests at {rate:.0f}/s over {arrivals[-1]:.2f} s, "
        f"{req_pairs:.3e} pair-evaluations")
    results = {}
    for name, streams, max_batch, prec in (("serial_fp64", 1, 1, "fp64"),
                                           ("continuous_fp64", 4, 64, "fp64"),
                                           ("continuous_fp32k", 4, 64, "fp32k")):
        srv = nqs.Server(HBM_BUDGET, streams=streams, max_batch=max_batch, precision=prec)
        for h, w in zip(hams, jobs):
            srv.add(h, w.n_samples)
        # warm-up: one request per job
        for h, p in zip(hams, payloads):
            srv.submit(h, *p[0])
        srv.drain(600.0)
        srv.poll()
        lat, wall = replay(srv, hams, payloads, arrivals, job_of)
        st = srv.stats()
        srv.close()
        results[name] = {
            "requests_per_s": n_req / wall,
            "pair_evals_per_s": req_pairs / wall,
            "p50_ms": float(np.percentile(lat, 50)) / 1e3,
            "p99_ms": float(np.percentile(lat, 99)) / 1e3,
            "mean_ms": float(lat.mean()) / 1e3,
            "wall_s": wall,
            "launches": st["launches"] - n_jobs if max_batch == 1 else st["launches"],
            "max_requests_in_flight": st["max_requests_in_flight"],
            "max_launches_in_flight": st["max_launches_in_flight"],
            "peak_admitted_GB": st["peak_bytes"] / 1e9,
        }
        log(f"{name}: {results[name]['requests_per_s']:.1f} req/s, p50 "
            f"{results[name]['p50_ms']:.1f} ms, p99 {results[name]['p99_ms']:.1f} ms, "
            f"in flight up to {st['max_requests_in_flight']} requests / "
            f"{st['max_launches_in_flight']} launches")
    for h in hams:
        h.sync()
        h.close()
    best = results["continuous_fp32k"]
    out = {
        "metric": "served E_loc requests/s with p50/p99 latency",
        "value": best["requests_per_s"],
        "unit": "requests/s",
        "n_gpus": 1, "steps": n_req, "warmup": n_jobs,
        "ms_per_step": 1e3 / best["requests_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+kahan/f64", "data": "synthetic",
        "config": {"workload": f"{n_jobs} synthetic VMC jobs (qubits 24..80, samples 1e3..2e5), "
                               f"Poisson arrivals {rate:.0f}/s, {n_req} requests, 64 GB budget",
                   "pair_evaluations": req_pairs},
        "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"],
        "modes": results,
        "throughput_vs_serial_fp64": best["requests_per_s"] / results["serial_fp64"]["requests_per_s"],
    }
    print(json.dumps(out), flush=True)
