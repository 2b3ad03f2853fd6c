"""Eq. 1 on the device (nqs_energy) against the oracle's exactly rounded
two-pass sums, at full batch sizes with geometric counts: the weighted mean
(re, im), the population variance and the sum of the counts.

The local energies are fixed synthetic arrays (the reduction does not care
where they come from): a molecule-like spread around a large mean, so that
the variance pass works against cancellation, and a heavy-tailed case.
Tolerances: mean within 1e-12 of sum w |E| / sum w, variance within 1e-12 of
its square (or of the variance itself where a heavy tail makes that the
larger); the count sum is an exact integer.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2506_23809_amd as nqs
import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-energy] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    nqs.load_library()
    return torch


@pytest.mark.parametrize("n", [65536, 262144, 262144 + 777])
@pytest.mark.parametrize("kind", ["molecular", "heavy_tail"])
def test_weighted_energy_matches_oracle(torch_dev, n, kind):
    torch = torch_dev
    rng = np.random.default_rng([41, n, len(kind)])
    w = W.geometric_weights(rng, n)
    w[rng.choice(n, n // 50, replace=False)] = 0  # unsampled rows carry no weight
    if kind == "molecular":
        e = rng.normal(-75.0, 4.0, n) + 1j * rng.normal(0.0, 0.3, n)
    else:
        e = rng.standard_cauchy(n) * 3.0 - 20.0 + 1j * rng.standard_cauchy(n)
    m_ref, v_ref, sw_ref = oracle.energy(w, e)
    wt = torch.from_numpy(w).cuda()
    et = torch.from_numpy(np.stack([e.real, e.imag], 1).copy()).cuda()
    say(f"{kind}, n = {n}")
    m, v, sw = nqs.energy(wt, et)
    scale = float(np.sum(w * np.abs(e)) / np.sum(w))
    say(f"|dmean| = {abs(m - m_ref):.3e}, |dvar| = {abs(v - v_ref):.3e}, scale {scale:.3e}")
    assert sw == sw_ref == float(w.sum())
    assert abs(m.real - m_ref.real) <= 1e-12 * scale
    assert abs(m.imag - m_ref.imag) <= 1e-12 * scale
    # a heavy tail makes the variance itself far larger than scale^2: its
    # rounding is relative to it then
    assert abs(v - v_ref) <= 1e-12 * max(scale * scale, v_ref)
    # fixed reduction order: a repeat gives the same bits
    m2, v2, sw2 = nqs.energy(wt, et)
    assert (m2, v2, sw2) == (m, v, sw)


def test_weighted_energy_of_a_device_eloc(torch_dev, workload_cache):
    """The full 40-qubit batch: E_loc from the library, counts from the
    workload, Eq. 1 on the device against the oracle applied to the same
    E_loc array."""
    torch = torch_dev
    wl = workload_cache(("workload", "nq40"))
    ham = nqs.Hamiltonian(wl.x, wl.z, wl.c, wl.n_qubits, wl.spin_masks)
    S = nqs.to_device_samples(wl.samples)
    la = torch.from_numpy(wl.log_amp).cuda()
    ph = torch.from_numpy(wl.phase).cuda()
    wt = torch.from_numpy(wl.weights).cuda()
    e = ham.eloc(S, la, ph, wt)
    m, v, sw = nqs.energy(wt, e)
    ham.sync()
    r = torch.view_as_real(e).cpu().numpy()
    el = r[:, 0] + 1j * r[:, 1]
    m_ref, v_ref, sw_ref = oracle.energy(wl.weights, el)
    scale = float(np.sum(wl.weights * np.abs(el)) / np.sum(wl.weights))
    say(f"nq40: E = {m.real:.10f}, var = {v:.6e}")
    assert sw == sw_ref
    assert abs(m - m_ref) <= 1e-12 * scale
    assert abs(v - v_ref) <= 1e-12 * scale * scale
    ham.close()
