"""The pair join (samples bucketed by the contents of max_flip + 1 qubit
blocks, pairs tested inside buckets) against the CPU oracle and against the
other strategies, through the C ABI.

Floating point within 1e-12 A(x) (FP64) or 1e-6 A(x) (FP32 with
compensation) of the oracle; hit counts equal the oracle's connected pairs;
debug dumps (lookup index of every (sample, group) pair, sign bit of every
evaluated term) bit-identical to the streaming kernel's.
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
FP32_TOL = 1e-6


def say(msg):
    print(f"[gpu-join] {msg}", flush=True)
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
    return r[:, 0] + 1j * r[:, 1], ham.stats(), ham.plan()


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
    return hit.cpu().numpy(), bits.cpu().numpy(), ham.plan()


@pytest.mark.parametrize("name,n", [("nq12", None), ("nq40", 4096), ("nq40", None),
                                    ("nq100", 4096)])
def test_join_agrees_with_the_oracle(torch_dev, name, n, workload_cache):
    w = workload_cache(("workload", name) if n is None else ("workload", name, n))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    ref, ab, nc = workload_cache(("oracle-full", w.name), lambda: oracle.eloc(
        w.n_qubits, w.x, w.z, w.c, w.samples, w.log_amp, w.phase))
    for precision, tol in (("fp64", TOL), ("fp32k", FP32_TOL)):
        say(f"{w.name}: join, {precision}")
        e, st, plan = _eval(torch_dev, ham, w.samples, w.log_amp, w.phase, "join", precision)
        say(f"plan {plan}, stats {st}")
        assert plan["join_blocks"] == 5 and plan["join_ran"] == 1
        assert st["enum_rounds"] == 0
        _parity(e, ref, ab, tol)
        assert st["hits"] == int(nc.sum()) - w.n_samples
        # every ordered pair inside a bucket is a candidate, every hit passed
        # the distance test first
        assert st["hits"] <= st["probes"] <= st["candidates"]
    ham.close()


@pytest.mark.parametrize("name,n", [("nq12", None), ("nq40", 1024), ("nq40", 8192)])
def test_join_dumps_equal_streaming(torch_dev, name, n, workload_cache):
    w = workload_cache(("workload", name) if n is None else ("workload", name, n))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    say(f"{w.name}: dumps of the join and of streaming")
    hs, bs, _ = _dump(torch_dev, ham, w.samples, w.log_amp, w.phase, "stream")
    hj, bj, plan = _dump(torch_dev, ham, w.samples, w.log_amp, w.phase, "join")
    assert plan["join_ran"] == 1
    assert np.array_equal(hs, hj)
    assert np.array_equal(bs, bj)
    # every sample finds itself (the diagonal); the hit-heavy 12-qubit set
    # and the larger 40-qubit batch also have partners
    assert (hj >= 0).sum() >= w.n_samples
    if w.n_samples != 1024:
        assert (hj >= 0).sum() > w.n_samples
    ham.close()


def test_join_closure_sets_and_word_boundary(torch_dev, workload_cache):
    """Hit-heavy sets (hundreds of partners per sample), flips on both sides
    of the 64-bit word boundary at 100 qubits."""
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from test_oracle_pins import closure_set
    for K, name in ((20, "nq40"), (50, "nq100")):
        w = workload_cache(("workload", name, 256))
        S = closure_set(K, K // 2, 2, 150, seed=K)
        rng = np.random.default_rng(4)
        la, ph = rng.normal(0, 0.5, S.shape[0]), rng.uniform(0, 2 * math.pi, S.shape[0])
        ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
        say(f"closure set {2 * K} qubits, {S.shape[0]} samples, join")
        ref, ab, nc = oracle.eloc(2 * K, w.x, w.z, w.c, S, la, ph)
        for precision, tol in (("fp64", TOL), ("fp32k", FP32_TOL)):
            e, st, plan = _eval(torch_dev, ham, S, la, ph, "join", precision)
            assert plan["join_ran"] == 1
            _parity(e, ref, ab, tol)
            assert st["hits"] == int(nc.sum()) - S.shape[0]
        ham.close()


def test_join_full_size_planted(torch_dev, workload_cache):
    """The 100-qubit table with 2^18 samples and planted neighbours of every
    flip kind: all rows against the full S x S oracle."""
    torch = torch_dev
    K, n_total = 50, 1 << 18
    w = workload_cache(("workload", "nq100", 256))
    rng = np.random.default_rng([21, K])
    S = workload_cache(("planted", K), lambda: W.planted_samples(rng, K, K // 2, K // 2, 200,
                                                                 n_total))
    la = np.random.default_rng([21, K, 3]).normal(0.0, 2.0, n_total)
    ph = np.random.default_rng([21, K, 4]).uniform(0.0, 2 * math.pi, n_total)
    ref, ab, nc = workload_cache(("planted-oracle", K), lambda: oracle.eloc(
        2 * K, w.x, w.z, w.c, S, la, ph))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    for strategy in ("auto", "join"):
        for precision, tol in (("fp64", TOL), ("fp32k", FP32_TOL)):
            say(f"100 qubits, {n_total} planted samples, {strategy}, {precision}")
            e, st, plan = _eval(torch, ham, S, la, ph, strategy, precision)
            say(f"plan {plan}, stats {st}")
            assert plan["join_ran"] == 1  # the cost model picks the join here
            assert st["hits"] == int(nc.sum()) - n_total
            _parity(e, ref, ab, tol)
    ham.close()


def test_join_duplicates_and_edges(torch_dev, workload_cache):
    torch = torch_dev
    w = workload_cache(("workload", "nq40", 4096))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    ham.set_tuning(strategy="join")
    la = torch.zeros(300, dtype=torch.float64, device="cuda")
    say("join: duplicate sample latched")
    s = w.samples[:300].copy()
    s[17] = s[250]
    ham.eloc(nqs.to_device_samples(s), la, la)
    with pytest.raises(nqs.NQSError) as ex:
        ham.sync()
    assert ex.value.code == nqs.NQS_E_DUPLICATE
    for n in (1, 2, 63, 65, 1000):
        say(f"join: n = {n}")
        e, st, plan = _eval(torch, ham, w.samples[:n], w.log_amp[:n], w.phase[:n], "join")
        ref, ab, nc = oracle.eloc(40, w.x, w.z, w.c, w.samples[:n], w.log_amp[:n], w.phase[:n])
        _parity(e, ref, ab)
        assert st["hits"] == int(nc.sum()) - n
    say("join: repeated calls give the same bits")
    S = nqs.to_device_samples(w.samples)
    la_t = torch.from_numpy(w.log_amp).cuda()
    ph_t = torch.from_numpy(w.phase).cuda()
    a = torch.view_as_real(ham.eloc(S, la_t, ph_t)).cpu().numpy()
    b = torch.view_as_real(ham.eloc(S, la_t, ph_t)).cpu().numpy()
    ham.sync()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    ham.close()


def test_join_stands_down_for_an_oversized_bucket(torch_dev, workload_cache):
    """Samples that all share the contents of one block: that bucket holds
    more than the sorter takes, so even a forced join leaves the batch to the
    enumeration; results still match the oracle."""
    torch = torch_dev
    w = workload_cache(("workload", "nq40", 256))
    rng = np.random.default_rng(77)
    # orbitals 0..3 (qubits 0..7, the first block) fixed occupied, the rest uniform
    K, n = 20, 9000
    rest = W.sector_samples(rng, K - 4, 6, 6, n)
    bits = np.zeros((n, 40), bool)
    bits[:, :8] = True
    bits[:, 8:] = W.unpack_bits(rest, 32)
    S = W.pack_bits(bits)
    la, ph = rng.normal(0, 1, n), rng.uniform(0, 2 * math.pi, n)
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    say(f"join with one bucket of {n} samples")
    e, st, plan = _eval(torch, ham, S, la, ph, "join")
    assert plan["join_ran"] == 0 and st["enum_rounds"] > 0
    rows = np.unique(rng.choice(n, 200, replace=False))
    ref, ab, _ = oracle.eloc_rows(40, w.x, w.z, w.c, S, la, ph, rows)
    _parity(e[rows], ref, ab)
    ham.close()


def test_join_general_table_without_spin_masks(torch_dev):
    """A non-molecular table (flips of up to 6 qubits, no spin masks, so no
    enumeration): the join against the oracle, and against streaming."""
    torch = torch_dev
    nq, T = 36, 4000
    rng = np.random.default_rng(36)
    xb = np.zeros((T, nq), bool)
    for t in range(T):
        k = rng.integers(0, 7)
        xb[t, rng.choice(nq, k, replace=False)] = True
    zb = rng.random((T, nq)) < 0.3
    for t in range(T):
        if np.sum(xb[t] & zb[t]) % 2:
            zb[t, np.nonzero(xb[t] & zb[t])[0][0]] = False
    x, z = W.pack_bits(xb), W.pack_bits(zb)
    c = rng.normal(size=T)
    base = W.pack_bits(rng.random((3000, nq)) < 0.5)
    extra = base[:600] ^ x[rng.integers(0, T, 600)]
    S = np.unique(np.concatenate([base, extra]), axis=0)
    S = S[rng.permutation(S.shape[0])]
    la, ph = rng.normal(0, 1, S.shape[0]), rng.uniform(0, 2 * math.pi, S.shape[0])
    ham = nqs.Hamiltonian(x, z, c, nq, None)
    say(f"general table, {nq} qubits, {S.shape[0]} samples")
    ref, ab, nc = oracle.eloc(nq, x, z, c, S, la, ph)
    e, st, plan = _eval(torch, ham, S, la, ph, "join")
    assert plan["join_blocks"] == 7 and plan["join_ran"] == 1
    _parity(e, ref, ab)
    has_diag = bool(np.any((x[:, 0] == 0) & (x[:, 1] == 0)))
    assert st["hits"] == int(nc.sum()) - (S.shape[0] if has_diag else 0)
    e2, _, _ = _eval(torch, ham, S, la, ph, "stream")
    _parity(e2, ref, ab)
    ham.close()


def test_join_integral_form(torch_dev, workload_cache):
    """The Slater-Condon form through the join: same hits and values as the
    Pauli table of the same integrals (oracle)."""
    w = workload_cache(("workload", "nq40", 4096))
    ham = nqs.Hamiltonian.from_integrals(w.h, w.eri)
    say("integral form, 40 qubits, join")
    e, st, plan = _eval(torch_dev, ham, w.samples, w.log_amp, w.phase, "join")
    ref, ab, nc = workload_cache(("oracle-full", w.name), lambda: oracle.eloc(
        w.n_qubits, w.x, w.z, w.c, w.samples, w.log_amp, w.phase))
    assert plan["join_ran"] == 1
    _parity(e, ref, ab)
    assert st["hits"] == int(nc.sum()) - w.n_samples
    ham.close()
