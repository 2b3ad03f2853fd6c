"""The two lookup strategies (group streaming, flip enumeration) against the
CPU oracle and against each other, through the C ABI.

Both evaluate Eq. 5 over the same hits with the same matrix elements; the
enumeration visits only each sample's spin-conserving singles and doubles.
Floating point: within 1e-12 * A(x) of the oracle.  Integers (hits, and
probes where the table holds every in-sector flip) and debug dumps: exact.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2506_23809_amd as nqs
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(msg):
    print(f"[gpu-enum] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    nqs.load_library()
    return torch


def _parity(e, ref, ab, tol=TOL):
    err = np.abs(e - ref)
    bad = err > tol * ab
    assert not bad.any(), f"{bad.sum()} rows off, worst {(err / np.maximum(ab, 1e-300)).max():.3e}"


def _eval(torch, ham, S_np, la, ph, strategy, precision="fp64"):
    ham.set_tuning(strategy=strategy)
    S = nqs.to_device_samples(S_np)
    la_t = torch.from_numpy(np.ascontiguousarray(la, dtype=np.float64)).cuda()
    ph_t = torch.from_numpy(np.ascontiguousarray(ph, dtype=np.float64)).cuda()
    e = ham.eloc(S, la_t, ph_t, precision=precision)
    ham.sync()
    r = torch.view_as_real(e).cpu().numpy()
    return r[:, 0] + 1j * r[:, 1], ham.stats()


def _dump(torch, ham, S_np, la, ph, strategy):
    ham.set_tuning(strategy=strategy)
    G, T, _ = ham.info()
    S = nqs.to_device_samples(S_np)
    la_t = torch.from_numpy(np.ascontiguousarray(la, dtype=np.float64)).cuda()
    ph_t = torch.from_numpy(np.ascontiguousarray(ph, dtype=np.float64)).cuda()
    hit = torch.full((S_np.shape[0], G), -7, dtype=torch.int32, device="cuda")
    bits = torch.zeros((S_np.shape[0], max((T + 31) // 32, 1)), dtype=torch.int32, device="cuda")
    ham.debug_dump(S, la_t, ph_t, hit, bits if T else None)
    ham.sync()
    return hit.cpu().numpy(), bits.cpu().numpy()


@pytest.mark.parametrize("name,n", [("nq12", None), ("nq40", 4096), ("nq100", 2048)])
def test_strategies_agree_with_the_oracle(torch_dev, name, n, workload_cache):
    w = workload_cache(("workload", name) if n is None else ("workload", name, n))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    ref, ab, nc = oracle.eloc(w.n_qubits, w.x, w.z, w.c, w.samples, w.log_amp, w.phase)
    out = {}
    for strategy in ("stream", "enum"):
        say(f"{w.name}: {strategy}")
        e, st = _eval(torch_dev, ham, w.samples, w.log_amp, w.phase, strategy)
        _parity(e, ref, ab)
        assert st["hits"] == int(nc.sum()) - w.n_samples
        # the device ran the strategy asked for
        assert (st["enum_rounds"] > 0) == (strategy == "enum")
        out[strategy] = st
    G, _, conn = W.closed_form_counts(w.K, w.n_alpha)
    assert out["enum"]["probes"] == w.n_samples * conn
    if G == ham.n_groups:  # every in-sector flip has a group: identical probe counts
        assert out["stream"]["probes"] == out["enum"]["probes"]
    # the enumeration's filter survivors are a subset of the same probes
    assert out["enum"]["candidates"] <= out["enum"]["probes"]
    ham.close()


@pytest.mark.parametrize("name,n", [("nq12", None), ("nq40", 1024)])
def test_dumps_identical(torch_dev, name, n, workload_cache):
    w = workload_cache(("workload", name) if n is None else ("workload", name, n))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    say(f"{w.name}: debug dumps of both strategies")
    hs, bs = _dump(torch_dev, ham, w.samples, w.log_amp, w.phase, "stream")
    he, be = _dump(torch_dev, ham, w.samples, w.log_amp, w.phase, "enum")
    assert np.array_equal(hs, he)
    assert np.array_equal(bs, be)
    assert (hs >= 0).sum() == (he >= 0).sum() > 0
    ham.close()


def test_closure_set_dump_and_values(torch_dev, workload_cache):
    """Hit-heavy: every sample has hundreds of partners in S, at 40 and 100
    qubits (flips on both sides of the 64-bit word boundary)."""
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from test_oracle_pins import closure_set
    for K, name in ((20, "nq40"), (50, "nq100")):
        w = workload_cache(("workload", name, 256))
        S = closure_set(K, K // 2, 2, 150, seed=K)
        rng = np.random.default_rng(4)
        la, ph = rng.normal(0, 0.5, S.shape[0]), rng.uniform(0, 2 * math.pi, S.shape[0])
        ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
        say(f"closure set {2 * K} qubits, {S.shape[0]} samples, enumeration")
        e, st = _eval(torch_dev, ham, S, la, ph, "enum")
        ref, ab, nc = oracle.eloc(2 * K, w.x, w.z, w.c, S, la, ph)
        _parity(e, ref, ab)
        assert st["hits"] == int(nc.sum()) - S.shape[0]
        if K == 20:
            sub = S[:300]
            hs, bs = _dump(torch_dev, ham, sub, la[:300], ph[:300], "stream")
            he, be = _dump(torch_dev, ham, sub, la[:300], ph[:300], "enum")
            assert np.array_equal(hs, he) and np.array_equal(bs, be)
        ham.close()


@pytest.mark.parametrize("filter_bits", [32, 64])
def test_filter_partitions(torch_dev, filter_bits, workload_cache):
    """More filter bits than one 128 KB bitmap holds: the samples are split
    into classes (2 or 4 partitions at 65536 samples), each partition probed
    by exactly its share of the flips."""
    w = workload_cache(("workload", "nq40"))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    ham.set_tuning(filter_bits=filter_bits, strategy="enum")
    say(f"{w.name}: enumeration with {filter_bits} filter bits per sample")
    S = nqs.to_device_samples(w.samples)
    la = torch_dev.from_numpy(w.log_amp).cuda()
    ph = torch_dev.from_numpy(w.phase).cuda()
    e = ham.eloc(S, la, ph)
    ham.sync()
    st = ham.stats()
    r = torch_dev.view_as_real(e).cpu().numpy()
    e = r[:, 0] + 1j * r[:, 1]
    ref, ab, nc = oracle.eloc(40, w.x, w.z, w.c, w.samples, w.log_amp, w.phase)
    _parity(e, ref, ab)
    _, _, conn = W.closed_form_counts(20, 10)
    assert st["probes"] == w.n_samples * conn
    assert st["hits"] == int(nc.sum()) - w.n_samples
    assert st["enum_rounds"] > 0
    # more bits per sample: fewer filter survivors than the one-bitmap run
    ham.set_tuning(filter_bits=16, strategy="enum")
    ham.eloc(S, la, ph)
    ham.sync()
    assert st["candidates"] < ham.stats()["candidates"]
    ham.close()


# occupations (n_alpha, n_beta) of a 12-orbital register: empty and full
# shells (no virtual or no occupied orbital in a spin), one electron or one
# hole, unequal spins
OCCUPATIONS = [(0, 6), (12, 5), (1, 11), (6, 6), (11, 0), (2, 9), (12, 12), (0, 0)]


@pytest.fixture(scope="module")
def k12():
    h, eri = W.integrals(np.random.default_rng([6, 1]), 12, 4.0)
    x, z, c = W.jw_terms(h, eri)
    return x, z, c


@pytest.mark.parametrize("na,nb", OCCUPATIONS)
def test_occupations(torch_dev, k12, na, nb):
    x, z, c = k12
    K, nq = 12, 24
    n_sector = math.comb(K, na) * math.comb(K, nb)
    n = min(n_sector, 3000)
    rng = np.random.default_rng([6, 2, na, nb])
    if n == n_sector:
        S = W.sector_states(K, na, nb)
    else:
        S = W.sector_samples(rng, K, na, nb, n)
    la, ph = rng.normal(0, 1, n), rng.uniform(0, 2 * math.pi, n)
    ham = nqs.Hamiltonian(x, z, c, nq, W.spin_masks(nq))
    say(f"24 qubits, {na} alpha + {nb} beta, {n} samples")
    ref, ab, nc = oracle.eloc(nq, x, z, c, S, la, ph)
    for strategy in ("enum", "stream"):
        e, st = _eval(torch_dev, ham, S, la, ph, strategy)
        _parity(e, ref, ab)
        assert st["hits"] == int(nc.sum()) - n
        assert (st["enum_rounds"] > 0) == (strategy == "enum")
    ham.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32k"])
def test_batch_mixing_strategies(torch_dev, precision):
    """One batch, jobs with either strategy: equal to single launches with the
    same tunings, bit for bit."""
    torch = torch_dev
    jobs = []
    # the 70000-sample job needs two filter partitions
    for j, (nq, n, strategy) in enumerate([(24, 1500, "enum"), (40, 3000, "stream"),
                                           (68, 2000, "enum"), (32, 900, "stream"),
                                           (72, 1200, "enum"), (24, 70000, "enum")]):
        K = nq // 2
        w = W.molecule([7, 100 + j], K, K // 2, K - K // 2, n, L=4.0, log_sigma=1.5,
                       name=f"mix-{j}")
        h = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
        h.set_tuning(strategy=strategy)
        jobs.append((w, h, nqs.to_device_samples(w.samples), torch.from_numpy(w.log_amp).cuda(),
                     torch.from_numpy(w.phase).cuda(),
                     torch.zeros((n, 2), dtype=torch.float64, device="cuda")))
    say(f"batch mixing strategies, {precision}")
    b = nqs.Batch([(h, S, la, ph, None, out) for (_, h, S, la, ph, out) in jobs],
                  precision=precision)
    b.launch()
    torch.cuda.synchronize()
    for w, h, S, la, ph, out in jobs:
        single = torch.view_as_real(h.eloc(S, la, ph, precision=precision)).cpu().numpy()
        h.sync()
        got = out.cpu().numpy()
        assert np.array_equal(single.view(np.uint64), got.view(np.uint64)), w.name
        rows = np.unique(np.random.default_rng(1).choice(w.n_samples, 48, replace=False))
        ref, ab, _ = oracle.eloc_rows(w.n_qubits, w.x, w.z, w.c, w.samples, w.log_amp, w.phase,
                                      rows)
        e = got[rows, 0] + 1j * got[rows, 1]
        _parity(e, ref, ab, tol=TOL if precision == "fp64" else 1e-6)
    b.close()
    for _, h, *_ in jobs:
        h.close()


def test_fp32_batch_keeps_integral_jobs_in_fp64(torch_dev, workload_cache):
    """An FP32+compensation batch evaluates integral-form jobs in FP64: their
    results equal an FP64 single launch bit for bit."""
    torch = torch_dev
    w1 = workload_cache(("workload", "nq40", 4096))
    w0 = workload_cache(("workload", "nq12"))
    sc = nqs.Hamiltonian.from_integrals(w1.h, w1.eri)
    pa = nqs.Hamiltonian(w0.x, w0.z, w0.c, 12, w0.spin_masks)
    jobs = []
    for h, w in ((sc, w1), (pa, w0)):
        jobs.append((h, nqs.to_device_samples(w.samples), torch.from_numpy(w.log_amp).cuda(),
                     torch.from_numpy(w.phase).cuda(), None,
                     torch.zeros((w.n_samples, 2), dtype=torch.float64, device="cuda")))
    say("fp32k batch with an integral-form job")
    for strategy in ("enum", "stream"):
        for h, *_ in jobs:
            h.set_tuning(strategy=strategy)
        b = nqs.Batch(jobs, precision="fp32k")
        b.launch()
        torch.cuda.synchronize()
        h, S, la, ph, _, out = jobs[0]
        single = torch.view_as_real(h.eloc(S, la, ph)).cpu().numpy()
        h.sync()
        assert np.array_equal(single.view(np.uint64), out.cpu().numpy().view(np.uint64)), strategy
        h, S, la, ph, _, out = jobs[1]
        single = torch.view_as_real(h.eloc(S, la, ph, precision="fp32k")).cpu().numpy()
        h.sync()
        assert np.array_equal(single.view(np.uint64), out.cpu().numpy().view(np.uint64)), strategy
        b.close()
    sc.close()
    pa.close()
