"""Serving leg of bench.py: synthetic VMC jobs issuing E_loc requests.

64 jobs are drawn from the batched-family distribution (qubits 24..80 at
half filling, samples log-uniform in [1e3, 2e5]); each keeps its Hamiltonian
resident and alternates between two sample batches (with their psi values).
Requests arrive as a Poisson process, each for a uniformly chosen job.  The
same arrival trace is replayed through three server configurations:

* serial FP64: one lane (one request on the device at a time, in arrival
  order: plain FP64 launches one after another);
* continuous FP64 and continuous FP32+compensation: four lanes, requests
  admitted as lanes free up and HBM allows (64 GB budget), overlapping on
  the device.

A sweep replays traces at increasing aggregate rates, the last submitting
every request at once (saturation: the throughput ceiling).  Reported per
point: completed requests per second, pair-evaluations per second and the
p50 / p99 latency from submission to completion.
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


MODES = (("serial_fp64", 1, "fp64"), ("continuous_fp64", 4, "fp64"),
         ("continuous_fp32k", 4, "fp32k"))


def run(args, log):
    import torch

    import paper_2506_23809_amd as nqs

    n_jobs = 64
    n_req = getattr(args, "requests", 0) or 2000
    rates = [float(r) for r in str(getattr(args, "rates", "") or "200,1000,2000,3000,4000,inf").split(",")]
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
    servers = {}
    for name, lanes, prec in MODES:
        srv = nqs.Server(HBM_BUDGET, streams=lanes, precision=prec)
        for h, w in zip(hams, jobs):
            srv.add(h, w.n_samples)
        # warm-up: one request per job
        for h, p in zip(hams, payloads):
            srv.submit(h, *p[0])
        srv.drain(600.0)
        srv.poll()
        servers[name] = srv
    sweep = []
    for rate in rates:
        arrivals, job_of = poisson_trace(n_req, rate if math.isfinite(rate) else 1e12, n_jobs)
        if not math.isfinite(rate):
            arrivals = np.zeros_like(arrivals)
        req_pairs = float(sum(pairs[j] for j in job_of))
        point = {"rate_per_s": rate if math.isfinite(rate) else "saturation",
                 "requests": n_req, "pair_evaluations": req_pairs}
        for name, lanes, prec in MODES:
            srv = servers[name]
            before = srv.stats()
            lat, wall = replay(srv, hams, payloads, arrivals, job_of)
            st = srv.stats()
            point[name] = {
                "requests_per_s": n_req / wall,
                "pair_evals_per_s": req_pairs / wall,
                "p50_ms": float(np.percentile(lat, 50)) / 1e3,
                "p99_ms": float(np.percentile(lat, 99)) / 1e3,
                "mean_ms": float(lat.mean()) / 1e3,
                "wall_s": wall,
                "requests_above_p99": int(np.sum(lat > np.percentile(lat, 99))),
                "launches": st["launches"] - before["launches"],
                "max_requests_in_flight": st["max_requests_in_flight"],
            }
            log(f"rate {point['rate_per_s']}: {name}: "
                f"{point[name]['requests_per_s']:.1f} req/s, p50 {point[name]['p50_ms']:.2f} ms, "
                f"p99 {point[name]['p99_ms']:.2f} ms")
        sweep.append(point)
    for srv in servers.values():
        srv.close()
    for h in hams:
        h.sync()
        h.close()
    sat = sweep[-1]
    best = sat["continuous_fp32k"]
    out = {
        "metric": "served E_loc requests/s with p50/p99 latency",
        "value": best["requests_per_s"],
        "unit": "requests/s",
        "n_gpus": 1, "steps": n_req, "warmup": n_jobs,
        "ms_per_step": 1e3 / best["requests_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+kahan/f64", "data": "synthetic",
        "config": {"workload": f"{n_jobs} synthetic VMC jobs (qubits 24..80, samples 1e3..2e5), "
                               f"Poisson arrivals at {rates} per s, {n_req} requests per point, "
                               f"64 GB budget, 4 lanes"},
        "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"],
        "sweep": sweep,
        "saturation_throughput_vs_serial_fp64": {
            name: sat[name]["requests_per_s"] / sat["serial_fp64"]["requests_per_s"]
            for name, _, _ in MODES},
    }
    print(json.dumps(out), flush=True)
