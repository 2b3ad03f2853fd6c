"""Batched persistent form, HIP-graph replay and autotuner, through the C ABI.

Batched results must equal single launches (bit for bit with the same
tuning) and the oracle within the FP64 tolerance.  Graph replays are checked
against eager results after eager work and synchronisation between replays.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2506_23809_amd as nqs
import workloads as W

pytestmark = pytest.mark.gpu

# (n_qubits, n_samples): one- and two-word masks, 32- and 64-bit sector
# fields, uneven sizes, an empty job
FAMILY = [(24, 1000), (36, 20000), (48, 3000), (64, 8000), (72, 2500), (28, 0), (40, 12000)]


def say(msg):
    print(f"[gpu-batched] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    nqs.load_library()
    return torch


@pytest.fixture(scope="module")
def family():
    out = []
    for j, (nq, n) in enumerate(FAMILY):
        K = nq // 2
        w = W.molecule([3, 100 + j], K, K // 2, K - K // 2, max(n, 1), L=4.0, log_sigma=2.0,
                       name=f"family-{j}-nq{nq}")
        if n == 0:
            w.samples = w.samples[:0]
            w.weights = w.weights[:0]
            w.log_amp = w.log_amp[:0]
            w.phase = w.phase[:0]
        out.append(w)
    return out


def _dev(torch, w):
    S = nqs.to_device_samples(w.samples) if w.n_samples else \
        torch.zeros((0, 2), dtype=torch.int64, device="cuda")
    la = torch.from_numpy(np.ascontiguousarray(w.log_amp)).cuda()
    ph = torch.from_numpy(np.ascontiguousarray(w.phase)).cuda()
    wt = torch.from_numpy(np.ascontiguousarray(w.weights)).cuda()
    out = torch.zeros((w.n_samples, 2), dtype=torch.float64, device="cuda")
    return S, la, ph, wt, out


def _check_rows(w, e, rows=64, tol=1e-12):
    if w.n_samples == 0:
        return
    sel = np.unique(np.random.default_rng(w.n_qubits).choice(w.n_samples, min(rows, w.n_samples),
                                                             replace=False))
    ref, ab, _ = oracle.eloc_rows(w.n_qubits, w.x, w.z, w.c, w.samples, w.log_amp, w.phase, sel)
    assert np.all(np.abs(e[sel] - ref) <= tol * ab)


def test_batch_equals_single_launches(torch_dev, family):
    torch = torch_dev
    hams = [nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks) for w in family]
    bufs = [_dev(torch, w) for w in family]
    say(f"batch of {len(family)} jobs: " + ", ".join(f"{w.n_qubits}q/{w.n_samples}" for w in family))
    b = nqs.Batch([(h, S, la, ph, wt, out) for h, (S, la, ph, wt, out) in zip(hams, bufs)])
    b.launch()
    torch.cuda.synchronize()
    batched = [out.cpu().numpy().copy() for (_, _, _, _, out) in bufs]
    stats_b = [h.stats() for h in hams]
    for h in hams:
        h.sync()
    say("single launches")
    for w, h, (S, la, ph, wt, out), eb, sb in zip(family, hams, bufs, batched, stats_b):
        if w.n_samples == 0:
            continue
        # the same plan as the batch (auto: the device picks the pair join or
        # the enumeration/streaming per job, the same way in both)
        e = h.eloc(S, la, ph, wt)
        h.sync()
        es = torch.view_as_real(e).cpu().numpy()
        assert np.array_equal(es.view(np.uint64), eb.view(np.uint64)), w.name
        ss = h.stats()
        assert ss["probes"] == sb["probes"] and ss["hits"] == sb["hits"]
        _check_rows(w, es[:, 0] + 1j * es[:, 1])
    b.close()
    for h in hams:
        h.close()


def test_batch_graph_replay(torch_dev, family):
    torch = torch_dev
    jobs = family[:4]
    hams = [nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks) for w in jobs]
    bufs = [_dev(torch, w) for w in jobs]
    side = torch.cuda.Stream()
    b = nqs.Batch([(h, S, la, ph, wt, out) for h, (S, la, ph, wt, out) in zip(hams, bufs)],
                  stream=side)
    say("eager reference")
    b.launch(side)
    side.synchronize()
    ref = [out.cpu().numpy().copy() for (*_, out) in bufs]
    say("capture")
    b.capture(side)
    side.synchronize()
    for rep in range(3):
        for (*_, out) in bufs:
            out.zero_()
        torch.cuda.synchronize()
        say(f"replay {rep}")
        b.replay(side)
        side.synchronize()
        for r, (*_, out) in zip(ref, bufs):
            assert np.array_equal(out.cpu().numpy().view(np.uint64), r.view(np.uint64))
        # eager work between replays
        b.launch(side)
        side.synchronize()
    # new samples in the same buffers: the replay sees them
    say("replay on new batch contents")
    new = []
    for j, (w, (S, la, ph, wt, out)) in enumerate(zip(jobs, bufs)):
        if w.n_samples == 0:
            new.append(None)
            continue
        rng = np.random.default_rng(77 + j)
        K = w.K
        s2 = W.sector_samples(rng, K, w.n_alpha, w.n_beta, w.n_samples)
        la2 = rng.normal(0, 1, w.n_samples)
        ph2 = rng.uniform(0, 2 * math.pi, w.n_samples)
        S.copy_(nqs.to_device_samples(s2))
        la.copy_(torch.from_numpy(la2))
        ph.copy_(torch.from_numpy(ph2))
        new.append((s2, la2, ph2))
    torch.cuda.synchronize()
    b.replay(side)
    side.synchronize()
    for w, h, nw, (*_, out) in zip(jobs, hams, new, bufs):
        if nw is None:
            continue
        s2, la2, ph2 = nw
        e = out.cpu().numpy()
        sel = np.arange(0, w.n_samples, max(1, w.n_samples // 48))
        r, ab, _ = oracle.eloc_rows(w.n_qubits, w.x, w.z, w.c, s2, la2, ph2, sel)
        assert np.all(np.abs(e[sel, 0] + 1j * e[sel, 1] - r) <= 1e-12 * ab)
    for h in hams:
        h.sync()
    b.close()
    for h in hams:
        h.close()


def test_batch_fp32_kahan(torch_dev, family):
    torch = torch_dev
    jobs = [w for w in family if w.n_samples]
    hams = [nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks) for w in jobs]
    bufs = [_dev(torch, w) for w in jobs]
    say("batch fp32k")
    b = nqs.Batch([(h, S, la, ph, wt, out) for h, (S, la, ph, wt, out) in zip(hams, bufs)],
                  precision="fp32k")
    b.launch()
    torch.cuda.synchronize()
    for w, (*_, wt, out) in zip(jobs, bufs):
        e = out.cpu().numpy()
        e = e[:, 0] + 1j * e[:, 1]
        _check_rows(w, e, rows=48, tol=1e-6)
    b.close()
    for h in hams:
        h.close()


def test_autotune_and_cache(torch_dev, tmp_path):
    torch = torch_dev
    w = W.workload("nq40", 4096)
    S, la, ph, wt, out = _dev(torch, w)
    cache = tmp_path / "tuning.json"
    h = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    say("autotune nq40-4096")
    best, ms = h.autotune(S, la, ph, out, cache_path=cache)
    assert best["threads"] in (256, 512, 1024) and ms > 0
    assert h.get_tuning() == best
    e = out.cpu().numpy()
    ref, ab, _ = oracle.eloc(40, w.x, w.z, w.c, w.samples, w.log_amp, w.phase)
    assert np.all(np.abs(e[:, 0] + 1j * e[:, 1] - ref) <= 1e-12 * ab)
    text = cache.read_text()
    assert '"threads"' in text and text.strip().startswith("{")
    h2 = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    best2, ms2 = h2.autotune(S, la, ph, out, cache_path=cache)
    assert ms2 == -1.0 and best2 == best
    # the tuned plan gives the oracle's result too
    e2 = torch.view_as_real(h2.eloc(S, la, ph)).cpu().numpy()
    assert np.all(np.abs(e2[:, 0] + 1j * e2[:, 1] - ref) <= 1e-12 * ab)
    with pytest.raises(nqs.NQSError):
        h2.set_tuning(threads=300)
    h.close()
    h2.close()
