"""Serving loop: continuous batching, admission by HBM footprint, and the same
result alone and in the mix (through the C ABI); served rows against the
CPU oracle (Eq. 5 over each request's sample set)."""
import sys

import numpy as np
import pytest

import oracle
import paper_2506_23809_amd as nqs
import workloads as W

pytestmark = pytest.mark.gpu

JOBS = [(24, 1500), (28, 4000), (32, 900), (36, 3000), (40, 5000), (28, 2500)]


def say(msg):
    print(f"[gpu-serving] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    nqs.load_library()
    return torch


@pytest.fixture(scope="module")
def setup(torch_dev):
    torch = torch_dev
    hams, payloads, host = [], [], []
    for j, (nq, n) in enumerate(JOBS):
        K = nq // 2
        w = W.molecule([5, 100 + j], K, K // 2, K - K // 2, n, L=4.0, log_sigma=1.5,
                       name=f"serve-{j}")
        h = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
        ps, hs = [], []
        for r in range(3):
            rng = np.random.default_rng([5, 100 + j, 20 + r])
            s = W.sector_samples(rng, K, w.n_alpha, w.n_beta, n)
            la = rng.normal(0, 1.5, n)
            ph = rng.uniform(0, 6.283185307179586, n)
            ps.append((nqs.to_device_samples(s), torch.from_numpy(la).cuda(),
                       torch.from_numpy(ph).cuda(), torch.from_numpy(w.weights).cuda(),
                       torch.zeros((n, 2), dtype=torch.float64, device="cuda")))
            hs.append((s, la, ph))
        hams.append(h)
        payloads.append(ps)
        host.append((w, hs))
    yield hams, payloads, host
    for h in hams:
        h.close()


def _alone(torch, h, p):
    S, la, ph, wt, _ = p
    e = h.eloc(S, la, ph, wt)
    h.sync()
    return torch.view_as_real(e).cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32k"])
def test_each_result_same_alone_and_in_the_mix(torch_dev, setup, precision):
    torch = torch_dev
    hams, payloads, host = setup
    srv = nqs.Server(8 * 1024 ** 3, streams=3, max_batch=8, precision=precision)
    for h, (nq, n) in zip(hams, JOBS):
        srv.add(h, n)
    say(f"{precision}: submitting {sum(len(p) for p in payloads)} requests at once")
    tickets = {}
    order = [(j, r) for r in range(3) for j in range(len(hams))]
    for j, r in order:
        tickets[srv.submit(hams[j], *payloads[j][r])] = (j, r)
    srv.drain(120.0)
    done = dict(srv.poll())
    st = srv.stats()
    say(f"stats {st}")
    assert set(done) == set(tickets) and all(us > 0 for us in done.values())
    assert st["completed"] == st["submitted"] == len(order) and st["rejected"] == 0
    assert st["max_requests_in_flight"] > 1       # batched in the mix
    assert st["launches"] < len(order)
    served = {(j, r): payloads[j][r][4].cpu().numpy().copy() for j, r in order}
    srv.close()
    for (j, r), e_mix in served.items():
        S, la, ph, wt, _ = payloads[j][r]
        # the server runs batches, which take the enumeration (never the pair
        # join): alone means the single launch with that strategy
        hams[j].set_tuning(strategy="enum")
        e = hams[j].eloc(S, la, ph, wt, precision=precision)
        hams[j].sync()
        hams[j].set_tuning(strategy="auto")
        e_alone = torch.view_as_real(e).cpu().numpy()
        assert np.array_equal(e_alone.view(np.uint64), e_mix.view(np.uint64)), (j, r)
        # and against the oracle on 32 sampled rows of every served request
        w, hs = host[j]
        s_np, la_np, ph_np = hs[r]
        rows = np.sort(np.random.default_rng([j, r]).choice(s_np.shape[0], 32, replace=False))
        ref, ab, _ = oracle.eloc_rows(w.n_qubits, w.x, w.z, w.c, s_np, la_np, ph_np, rows)
        got = e_mix[rows, 0] + 1j * e_mix[rows, 1]
        tol = 1e-12 if precision == "fp64" else 1e-6
        err = np.abs(got - ref)
        assert np.all(err <= tol * ab), (j, r, float(np.max(err / ab)))


def test_admission_respects_the_budget(torch_dev, setup):
    torch = torch_dev
    hams, payloads, _ = setup
    # tables of all handles are resident; leave room for exactly one request
    probe = nqs.Server(1 << 40, streams=1, max_batch=1)
    resident = []
    for h, (nq, n) in zip(hams, JOBS):
        before = probe.stats()["resident_bytes"]
        probe.add(h, n)
        resident.append(probe.stats()["resident_bytes"] - before)
    probe.close()
    footprint = [56 * n + (h.info()[2] - t) for h, (nq, n), t in zip(hams, JOBS, resident)]
    budget = sum(resident) + max(footprint) + 1
    assert budget < sum(resident) + 2 * min(footprint)
    srv = nqs.Server(budget, streams=4, max_batch=8)
    for h, (nq, n) in zip(hams, JOBS):
        srv.add(h, n)
    say(f"budget {budget} bytes: one request at a time")
    for j in range(len(hams)):
        srv.submit(hams[j], *payloads[j][0])
    srv.drain(120.0)
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == len(hams)
    assert st["max_requests_in_flight"] == 1
    assert st["peak_bytes"] <= budget
    srv.close()
    # a request that can never fit is rejected at submission
    tiny = nqs.Server(sum(resident) + 1024, streams=1, max_batch=1)
    for h, (nq, n) in zip(hams, JOBS):
        tiny.add(h, n)
    with pytest.raises(nqs.NQSError) as ex:
        tiny.submit(hams[0], *payloads[0][0])
    assert ex.value.code == nqs.NQS_E_NOMEM
    assert tiny.stats()["rejected"] == 1
    tiny.close()
    with pytest.raises(nqs.NQSError):
        nqs.Server(0)
