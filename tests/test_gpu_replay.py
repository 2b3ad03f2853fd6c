"""Repeated evaluations with the same arguments are replayed as one captured
graph; every replay must equal an eager evaluation of the same inputs, bit
for bit, with the inputs rewritten in place and eager device work and
synchronisations between the replays.
"""
import os
import sys

import numpy as np
import pytest

import paper_2506_23809_amd as nqs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-replay] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    nqs.load_library()
    return torch


def _eager_handle(w):
    old = os.environ.get("NQS_EVAL_GRAPHS")
    os.environ["NQS_EVAL_GRAPHS"] = "0"
    try:
        return nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    finally:
        if old is None:
            del os.environ["NQS_EVAL_GRAPHS"]
        else:
            os.environ["NQS_EVAL_GRAPHS"] = old


@pytest.mark.parametrize("name,n", [("nq40", 4096), ("nq100", 3000)])
@pytest.mark.parametrize("precision", ["fp64", "fp32k"])
def test_replays_equal_eager(torch_dev, workload_cache, name, n, precision):
    torch = torch_dev
    w = workload_cache(("workload", name, n))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    ref = _eager_handle(w)
    S = nqs.to_device_samples(w.samples)
    la = torch.from_numpy(w.log_amp.copy()).cuda()
    ph = torch.from_numpy(w.phase.copy()).cuda()
    wt = torch.from_numpy(w.weights).cuda()
    out = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(17)
    profiled = []
    for r in range(6):
        say(f"{name} n={n} {precision} round {r}")
        # new amplitudes in the same buffers, then eager work of torch's own
        la.copy_(torch.from_numpy(rng.normal(0.0, 2.0, n)))
        ph.copy_(torch.from_numpy(rng.uniform(0.0, 2 * np.pi, n)))
        junk = (la * 2.0).sum().item()
        assert np.isfinite(junk)
        if r == 3:
            ham.profile(True)
        ham.eloc_into(out, S, la, ph, wt, precision=precision)
        ham.sync()
        got = out.cpu().numpy().copy()
        if r >= 3:
            # profiled calls run eagerly: every call times its own kernels
            ms = ham.last_kernel_ms()
            assert ms[1] > 0.0, ms
            profiled.append(tuple(ms))
        e = ref.eloc(S, la, ph, wt, precision=precision)
        ref.sync()
        want = torch.view_as_real(e).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (name, precision, r)
        m_got = nqs.energy(wt, out)
        m_want = nqs.energy(wt, torch.view_as_real(e).contiguous())
        assert m_got[0] == m_want[0] and m_got[1] == m_want[1], (m_got, m_want)
    ham.profile(False)
    # three calls, three measurements (not one replayed set of timestamps);
    # a single stage of a small batch can repeat its duration to the tick, so
    # the stages are compared together
    assert len(set(profiled)) > 1, profiled
    # a different batch size in between: eager again, then replays again
    k = n // 2
    out2 = torch.empty((k, 2), dtype=torch.float64, device="cuda")
    for r in range(3):
        ham.eloc_into(out2, S[:k], la[:k], ph[:k], wt[:k], precision=precision)
        ham.sync()
        e = ref.eloc(S[:k], la[:k], ph[:k], wt[:k], precision=precision)
        ref.sync()
        want = torch.view_as_real(e).cpu().numpy()
        assert np.array_equal(out2.cpu().numpy().view(np.uint64), want.view(np.uint64)), r
    ham.close()
    ref.close()
