"""Integral form (Slater-Condon evaluator) against the CPU oracle, which works
from the Jordan-Wigner Pauli table of the same integrals: two representations
of one Hamiltonian must give the same local energies."""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2506_23809_amd as nqs
import workloads as W
from oracle import dense

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-integrals] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    nqs.load_library()
    return torch


def _run(torch, ham, S_np, la, ph, dump=False):
    S = nqs.to_device_samples(S_np)
    la_t = torch.from_numpy(np.ascontiguousarray(la)).cuda()
    ph_t = torch.from_numpy(np.ascontiguousarray(ph)).cuda()
    if dump:
        G, T, _ = ham.info()
        hit = torch.full((S_np.shape[0], G), -7, dtype=torch.int32, device="cuda")
        e = ham.debug_dump(S, la_t, ph_t, hit_idx=hit)
        ham.sync()
        return torch.view_as_real(e).cpu().numpy(), hit.cpu().numpy()
    e = ham.eloc(S, la_t, ph_t)
    ham.sync()
    r = torch.view_as_real(e).cpu().numpy()
    return r[:, 0] + 1j * r[:, 1], ham.stats()


def test_nq12_random_psi_and_lookups(torch_dev, workload_cache):
    w = workload_cache(("workload", "nq12"))
    say("nq12 integral form")
    sc = nqs.Hamiltonian.from_integrals(w.h, w.eri)
    pa = nqs.Hamiltonian(w.x, w.z, w.c, 12, w.spin_masks)
    assert sc.n_groups == pa.n_groups == 286 and sc.n_terms == 0
    e, st = _run(torch_dev, sc, w.samples, w.log_amp, w.phase)
    ref, ab, nc = oracle.eloc(12, w.x, w.z, w.c, w.samples, w.log_amp, w.phase)
    assert np.all(np.abs(e - ref) <= 1e-12 * ab)
    assert st["hits"] == int(nc.sum()) - 400 and st["terms"] == 0
    _, hit_sc = _run(torch_dev, sc, w.samples, w.log_amp, w.phase, dump=True)
    _, hit_pa = _run(torch_dev, pa, w.samples, w.log_amp, w.phase, dump=True)
    assert np.array_equal(hit_sc, hit_pa)
    with pytest.raises(nqs.NQSError):
        S = nqs.to_device_samples(w.samples)
        z = torch_dev.zeros(400, dtype=torch_dev.float64, device="cuda")
        sc.eloc(S, z, z, precision="fp32k")
    sc.close()
    pa.close()


def test_nq12_ground_state(torch_dev, workload_cache):
    w = workload_cache(("workload", "nq12"))
    E0, v, _ = dense.sector_ground_state(w.h, w.eri, w.samples)
    sc = nqs.Hamiltonian.from_integrals(w.h, w.eri)
    e, _ = _run(torch_dev, sc, w.samples, np.log(np.abs(v)), np.where(v < 0, math.pi, 0.0))
    keep = np.abs(v) >= 1e-4 * np.abs(v).max()
    assert np.abs(e[keep] - E0).max() <= 1e-10
    sc.close()


@pytest.mark.parametrize("name,n", [("nq40", 4096), ("nq100", 2048)])
def test_uniform_batches(torch_dev, name, n, workload_cache):
    w = workload_cache(("workload", name, n))
    say(f"{w.name} integral form")
    sc = nqs.Hamiltonian.from_integrals(w.h, w.eri)
    pa = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    e, st = _run(torch_dev, sc, w.samples, w.log_amp, w.phase)
    ref, ab, nc = oracle.eloc(w.n_qubits, w.x, w.z, w.c, w.samples, w.log_amp, w.phase)
    assert np.all(np.abs(e - ref) <= 1e-12 * ab)
    _, st_pa = _run(torch_dev, pa, w.samples, w.log_amp, w.phase)
    # the flip table holds every spin-conserving flip; the Pauli table may lack
    # the few groups whose merged coefficients fell below the drop threshold
    assert st["probes"] >= st_pa["probes"] and st["hits"] >= st_pa["hits"]
    b_sc, b_pa = sc.info()[2], pa.info()[2]
    say(f"{w.name}: device bytes integral form {b_sc}, Pauli form {b_pa}")
    assert b_sc < b_pa
    sc.close()
    pa.close()


@pytest.mark.parametrize("K,n,L,name", [(20, 10, 4.0, "nq40"), (50, 25, 6.0, "nq100")])
def test_closure_sets(torch_dev, K, n, L, name, workload_cache):
    w = workload_cache(("workload", name, 256))
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from test_oracle_pins import closure_set
    S = closure_set(K, n, 2, 150, seed=K)
    rng = np.random.default_rng(4)
    la, ph = rng.normal(0, 0.5, S.shape[0]), rng.uniform(0, 2 * math.pi, S.shape[0])
    say(f"closure set {2 * K} qubits, {S.shape[0]} samples, integral form")
    sc = nqs.Hamiltonian.from_integrals(w.h, w.eri)
    e, _ = _run(torch_dev, sc, S, la, ph)
    ref, ab, _ = oracle.eloc(2 * K, w.x, w.z, w.c, S, la, ph)
    assert np.all(np.abs(e - ref) <= 1e-12 * ab)
    sc.close()


def test_batch_mixes_both_forms(torch_dev, workload_cache):
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
    b = nqs.Batch(jobs)
    b.launch()
    torch.cuda.synchronize()
    for h, S, la, ph, _, out in jobs:
        h.set_tuning(strategy="enum")  # the strategy a batch runs
        single = torch.view_as_real(h.eloc(S, la, ph)).cpu().numpy()
        h.sync()
        assert np.array_equal(single.view(np.uint64), out.cpu().numpy().view(np.uint64))
    b.close()
    sc.close()
    pa.close()
