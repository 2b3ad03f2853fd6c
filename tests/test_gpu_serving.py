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


def _check_oracle(host, j, r, e_mix, precision):
    """32 sampled rows of a served request against the oracle (Eq. 5 over
    that request's sample set)."""
    w, hs = host[j]
    s_np, la_np, ph_np = hs[r]
    rows = np.sort(np.random.default_rng([j, r]).choice(s_np.shape[0], 32, replace=False))
    ref, ab, _ = oracle.eloc_rows(w.n_qubits, w.x, w.z, w.c, s_np, la_np, ph_np, rows)
    got = e_mix[rows, 0] + 1j * e_mix[rows, 1]
    tol = 1e-12 if precision == "fp64" else 1e-6
    err = np.abs(got - ref)
    assert np.all(err <= tol * ab), (j, r, float(np.max(err / ab)))


@pytest.mark.parametrize("precision", ["fp64", "fp32k"])
def test_each_result_same_alone_and_in_the_mix(torch_dev, setup, precision):
    torch = torch_dev
    hams, payloads, host = setup
    srv = nqs.Server(8 * 1024 ** 3, streams=3, precision=precision)
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
    assert st["max_requests_in_flight"] > 1       # requests overlap on the lanes
    assert st["launches"] == len(order)           # one launch per request
    served = {(j, r): payloads[j][r][4].cpu().numpy().copy() for j, r in order}
    srv.close()
    for (j, r), e_mix in served.items():
        S, la, ph, wt, _ = payloads[j][r]
        # alone: the single launch (a lane takes the same plan)
        e = hams[j].eloc(S, la, ph, wt, precision=precision)
        hams[j].sync()
        e_alone = torch.view_as_real(e).cpu().numpy()
        assert np.array_equal(e_alone.view(np.uint64), e_mix.view(np.uint64)), (j, r)
        _check_oracle(host, j, r, e_mix, precision)


def test_requests_of_one_handle_overlap(torch_dev, setup):
    """Several requests for the same Hamiltonian at once: each lane has its
    own scratch, so they run together; each equals its single launch."""
    torch = torch_dev
    hams, payloads, host = setup
    j = 4  # 40 qubits, 5000 samples
    h = hams[j]
    srv = nqs.Server(8 * 1024 ** 3, streams=4)
    srv.add(h, JOBS[j][1])
    # three sample batches, each submitted twice into separate outputs
    reqs = []
    for r in range(3):
        for _ in range(2):
            S, la, ph, wt, _ = payloads[j][r]
            out = torch.full((S.shape[0], 2), float("nan"), dtype=torch.float64, device="cuda")
            reqs.append((r, out, srv.submit(h, S, la, ph, wt, out)))
    say(f"{len(reqs)} requests for one handle")
    srv.drain(120.0)
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == len(reqs)
    assert st["max_requests_in_flight"] > 1
    srv.close()
    for r, out, _ in reqs:
        S, la, ph, wt, _ = payloads[j][r]
        e_alone = torch.view_as_real(h.eloc(S, la, ph, wt)).cpu().numpy()
        h.sync()
        got = out.cpu().numpy()
        assert np.array_equal(e_alone.view(np.uint64), got.view(np.uint64)), r
        _check_oracle(host, j, r, got, "fp64")


def test_served_request_errors_are_latched_on_its_handle(torch_dev, setup):
    """A served request with a repeated sample: the server completes it and
    goes on; nqs_sync on that handle reports the duplicate; the next request
    on the same lane is correct."""
    torch = torch_dev
    hams, payloads, host = setup
    j = 0
    h = hams[j]
    srv = nqs.Server(8 * 1024 ** 3, streams=1)
    srv.add(h, JOBS[j][1])
    S, la, ph, wt, _ = payloads[j][0]
    bad = S.clone()
    bad[5] = bad[77]
    out = torch.zeros((S.shape[0], 2), dtype=torch.float64, device="cuda")
    say("served request with a duplicate sample")
    srv.submit(h, bad, la, ph, wt, out)
    srv.drain(60.0)
    with pytest.raises(nqs.NQSError) as ex:
        h.sync()
    assert ex.value.code == nqs.NQS_E_DUPLICATE
    h.sync()  # reported once
    out2 = torch.zeros((S.shape[0], 2), dtype=torch.float64, device="cuda")
    srv.submit(h, S, la, ph, wt, out2)
    srv.drain(60.0)
    h.sync()
    srv.close()
    _check_oracle(host, j, 0, out2.cpu().numpy(), "fp64")


def test_admission_respects_the_budget(torch_dev, setup):
    torch = torch_dev
    hams, payloads, _ = setup
    # the resident data: every table plus four lanes' scratch
    probe = nqs.Server(1 << 40, streams=4)
    for h, (nq, n) in zip(hams, JOBS):
        probe.add(h, n)
    resident = probe.stats()["resident_bytes"]
    probe.close()
    # the three largest requests: any two together exceed the headroom
    big = [k for k, (nq, n) in enumerate(JOBS) if n >= 3000]
    fp = [56 * JOBS[k][1] for k in big]
    budget = resident + max(fp) + 1
    assert 2 * min(fp) > max(fp) + 1
    srv = nqs.Server(budget, streams=4)
    for h, (nq, n) in zip(hams, JOBS):
        srv.add(h, n)
    assert srv.stats()["resident_bytes"] == resident
    say(f"budget {budget} bytes: one request at a time")
    for k in big:
        srv.submit(hams[k], *payloads[k][0])
    srv.drain(120.0)
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == len(big)
    assert st["max_requests_in_flight"] == 1
    assert st["peak_bytes"] <= budget
    srv.close()
    # a request that can never fit is rejected at submission
    tiny = nqs.Server(resident + 1024, streams=4)
    for h, (nq, n) in zip(hams, JOBS):
        tiny.add(h, n)
    with pytest.raises(nqs.NQSError) as ex:
        tiny.submit(hams[0], *payloads[0][0])
    assert ex.value.code == nqs.NQS_E_NOMEM
    assert tiny.stats()["rejected"] == 1
    # and so is one larger than its handle was registered for
    S, la, ph, wt, out = payloads[1][0]
    small = nqs.Server(1 << 40, streams=1)
    small.add(hams[1], 100)
    with pytest.raises(nqs.NQSError) as ex:
        small.submit(hams[1], S, la, ph, wt, out)
    assert ex.value.code == nqs.NQS_E_ARG
    small.close()
    tiny.close()
    with pytest.raises(nqs.NQSError):
        nqs.Server(0)
