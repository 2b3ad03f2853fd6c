"""nqs_eloc_energy: one VMC step's E_loc (Eq. 5) and Eq. 1 (§II-A) over it
in one launch sequence.

Checked on the full workloads (12 qubits with its ragged 400 samples, 40
qubits at 65,536 samples in 256-sample finish blocks, 100 qubits at 262,144
samples in 1024-sample blocks), eagerly and through the replayed graph:
  * E_loc is bit-identical to nqs_eloc_eval's on the same arguments;
  * the energy, variance and count sum agree with the oracle's exactly
    rounded sums over that E_loc (same tolerances as nqs_energy's tests:
    1e-12 of sum w |E| / sum w for the mean, of its square for the
    variance) and with nqs_energy over the same array;
  * repeated calls give identical bits;
  * device-detected errors come back from the call itself, and a clean
    call afterwards succeeds;
  * after a call that ran the pair join, the next one launches only the
    join's kernels: when the device declines the join for new contents of
    the same buffers, the call evaluates again with every launch and its
    result still equals nqs_eloc_eval's;
  * such a launch carries no hash build, yet a negative count or a bit
    beyond the register still fails the call (the grouping checks them).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2506_23809_amd as nqs
import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-eloc-energy] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    nqs.load_library()
    return torch


def _upload(torch, wl):
    S = nqs.to_device_samples(wl.samples)
    la = torch.from_numpy(wl.log_amp).cuda()
    ph = torch.from_numpy(wl.phase).cuda()
    wt = torch.from_numpy(wl.weights).cuda()
    return S, la, ph, wt


@pytest.mark.parametrize("name,precision", [("nq12", "fp64"), ("nq40", "fp64"),
                                            ("nq40", "fp32k"), ("nq100", "fp64")])
def test_eloc_energy_matches_eval_and_oracle(torch_dev, workload_cache, name, precision):
    torch = torch_dev
    wl = workload_cache(("workload", name))
    n = wl.samples.shape[0]
    ham = nqs.Hamiltonian(wl.x, wl.z, wl.c, wl.n_qubits, wl.spin_masks)
    S, la, ph, wt = _upload(torch, wl)
    say(f"{name} {precision}: n = {n}, reference evaluation")
    ref = torch.view_as_real(ham.eloc(S, la, ph, wt, precision=precision)).cpu().numpy()
    ham.sync()
    out = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    results = []
    for r in range(4):
        # eager (new arguments), eager (remembered), captured, replayed
        say(f"{name} {precision}: call {r}")
        out.fill_(float("nan"))
        results.append(ham.eloc_energy_into(out, S, la, ph, wt, precision=precision))
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (name, precision, r)
    assert all(res == results[0] for res in results), results
    m, v, sw = results[0]
    el = got[:, 0] + 1j * got[:, 1]
    m_ref, v_ref, sw_ref = oracle.energy(wl.weights, el)
    scale = float(np.sum(wl.weights * np.abs(el)) / np.sum(wl.weights))
    say(f"{name} {precision}: E = {m.real:.10f} (oracle {m_ref.real:.10f}), var = {v:.6e}")
    assert sw == sw_ref == float(wl.weights.sum())
    assert abs(m.real - m_ref.real) <= 1e-12 * scale
    assert abs(m.imag - m_ref.imag) <= 1e-12 * scale
    assert abs(v - v_ref) <= 1e-12 * max(scale * scale, v_ref)
    m2, v2, sw2 = nqs.energy(wt, out)
    assert sw2 == sw
    assert abs(m2 - m) <= 1e-12 * scale
    assert abs(v2 - v) <= 1e-12 * max(scale * scale, v)
    ham.close()


def test_eloc_energy_errors(torch_dev, workload_cache):
    torch = torch_dev
    wl = workload_cache(("workload", "nq12"))
    ham = nqs.Hamiltonian(wl.x, wl.z, wl.c, 12, wl.spin_masks)
    n = 50
    la = torch.zeros(n, dtype=torch.float64, device="cuda")
    ph = torch.zeros(n, dtype=torch.float64, device="cuda")
    wt = torch.ones(n, dtype=torch.int64, device="cuda")
    out = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    S = nqs.to_device_samples(wl.samples[:n])
    say("errors: duplicate sample, from the call itself")
    s = wl.samples[:n].copy()
    s[7] = s[31]
    with pytest.raises(nqs.NQSError) as ex:
        ham.eloc_energy_into(out, nqs.to_device_samples(s), la, ph, wt)
    assert ex.value.code == nqs.NQS_E_DUPLICATE
    say("errors: a clean call afterwards")
    m, v, sw = ham.eloc_energy_into(out, S, la, ph, wt)
    assert sw == float(n)
    ham.sync()  # nothing left latched
    say("errors: all counts zero")
    with pytest.raises(nqs.NQSError) as ex:
        ham.eloc_energy_into(out, S, la, ph, torch.zeros_like(wt))
    assert ex.value.code == nqs.NQS_E_ARG
    say("errors: empty batch")
    with pytest.raises(nqs.NQSError) as ex:
        ham.eloc_energy_into(out[:0], S[:0], la[:0], ph[:0], wt[:0])
    assert ex.value.code == nqs.NQS_E_ARG
    ham.close()


def test_join_only_launch_recovers_when_the_join_is_declined(torch_dev, workload_cache):
    torch = torch_dev
    w = workload_cache(("workload", "nq40", 256))
    rng = np.random.default_rng(91)
    n = 9000
    # spread samples of the 40-qubit sector: the device runs the join
    spread = W.sector_samples(rng, 20, 10, 10, n)
    # the same sector with the first block's qubits always occupied: one
    # bucket holds every sample, the join cannot run
    rest = W.sector_samples(rng, 16, 6, 6, n)
    bits = np.zeros((n, 40), bool)
    bits[:, :8] = True
    bits[:, 8:] = W.unpack_bits(rest, 32)
    clustered = W.pack_bits(bits)
    la = torch.from_numpy(rng.normal(0.0, 1.0, n)).cuda()
    ph = torch.from_numpy(rng.uniform(0.0, 2 * math.pi, n)).cuda()
    wt = torch.from_numpy(rng.integers(1, 5, n).astype(np.int64)).cuda()
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    ref_ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    S = nqs.to_device_samples(spread)
    out = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    for label, contents, join_ran in (("spread", spread, 1), ("spread", spread, 1),
                                      ("spread", spread, 1), ("clustered", clustered, 0),
                                      ("clustered", clustered, 0), ("spread", spread, 1)):
        say(f"join-only launch: {label}")
        S.copy_(nqs.to_device_samples(contents))
        ref = torch.view_as_real(ref_ham.eloc(S, la, ph, wt)).cpu().numpy()
        ref_ham.sync()
        assert ref_ham.plan()["join_ran"] == join_ran
        out.fill_(float("nan"))
        m, v, sw = ham.eloc_energy_into(out, S, la, ph, wt)
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), label
        m2, v2, sw2 = nqs.energy(wt, out)
        scale = float(np.sum(np.abs(got[:, 0] + 1j * got[:, 1])) / n)
        assert sw == sw2 and abs(m - m2) <= 1e-12 * scale
        assert ham.plan()["join_ran"] == join_ran
    ham.close()
    ref_ham.close()


def test_join_only_launch_still_checks_the_samples(torch_dev, workload_cache):
    """A launch that only joins carries no hash build: the grouping makes
    its checks.  After calls that chose the join (so that the next one
    launches the join alone), a negative count and then a bit beyond the
    register must still come back as NQS_E_RANGE from the call itself, and a
    clean call afterwards must match nqs_eloc_eval."""
    torch = torch_dev
    w = workload_cache(("workload", "nq40", 256))
    rng = np.random.default_rng(93)
    n = 9000
    spread = W.sector_samples(rng, 20, 10, 10, n)
    la = torch.from_numpy(rng.normal(0.0, 1.0, n)).cuda()
    ph = torch.from_numpy(rng.uniform(0.0, 2 * math.pi, n)).cuda()
    wt = torch.from_numpy(rng.integers(1, 5, n).astype(np.int64)).cuda()
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    S = nqs.to_device_samples(spread)
    out = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    for r in range(3):
        say(f"checks in join-only launches: clean call {r}")
        ham.eloc_energy_into(out, S, la, ph, wt)
        assert ham.plan()["join_ran"] == 1
    say("checks in join-only launches: a negative count")
    bad_w = wt.clone()
    bad_w[4321] = -1
    wt.copy_(bad_w)
    with pytest.raises(nqs.NQSError) as ex:
        ham.eloc_energy_into(out, S, la, ph, wt)
    assert ex.value.code == nqs.NQS_E_RANGE
    wt[4321] = 2
    say("checks in join-only launches: a bit beyond the register")
    bad = spread.copy()
    bad[777, 0] |= np.uint64(1) << np.uint64(45)
    S.copy_(nqs.to_device_samples(bad))
    with pytest.raises(nqs.NQSError) as ex:
        ham.eloc_energy_into(out, S, la, ph, wt)
    assert ex.value.code == nqs.NQS_E_RANGE
    say("checks in join-only launches: clean again")
    S.copy_(nqs.to_device_samples(spread))
    ref = torch.view_as_real(ham.eloc(S, la, ph, wt)).cpu().numpy()
    ham.sync()
    out.fill_(float("nan"))
    ham.eloc_energy_into(out, S, la, ph, wt)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), ref.view(np.uint64))
    ham.close()
