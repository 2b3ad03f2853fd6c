"""Full-size batches whose enumeration filter is split into 8 class
partitions, with planted neighbours so that every flip kind (alpha and beta
singles, alpha-alpha, beta-beta and alpha-beta doubles) produces hits across
partitions.

At 2^18 samples the library's default plan takes 32 filter bits per sample,
which needs 8 partitions of 128 KB: a flip that changes a beta orbital moves
its target to another sample class, so a wrong class route would drop hits.
Every row is compared with the full S x S oracle (FP64 within 1e-12 A(x),
FP32 with compensation within 1e-6 A(x) and 1e-6 Ha on Re <E>), and the hit
count must equal the oracle's connected pairs.
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
ENERGY_TOL_HA = 1e-6


def say(msg):
    print(f"[gpu-partitions] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    nqs.load_library()
    return torch


def _parity(e, ref, ab, tol):
    err = np.abs(e - ref)
    bad = err > tol * ab
    assert not bad.any(), f"{bad.sum()} rows off, worst {(err / np.maximum(ab, 1e-300)).max():.3e}"


@pytest.mark.parametrize("name,K,filter_bits", [("nq100", 50, 0), ("nq40", 20, 0),
                                                ("nq40", 20, 64)])
def test_eight_partitions_planted_hits(torch_dev, name, K, filter_bits, workload_cache):
    torch = torch_dev
    w = workload_cache(("workload", name, 256))  # the table; the batch is drawn below
    n_total = 1 << 18
    rng = np.random.default_rng([21, K])
    S = workload_cache(("planted", K), lambda: W.planted_samples(rng, K, K // 2, K // 2, 200,
                                                                 n_total))
    la = np.random.default_rng([21, K, 3]).normal(0.0, 2.0, n_total)
    ph = np.random.default_rng([21, K, 4]).uniform(0.0, 2 * math.pi, n_total)
    ref, ab, nc = workload_cache(("planted-oracle", K), lambda: oracle.eloc(
        2 * K, w.x, w.z, w.c, S, la, ph))
    n_hits = int(nc.sum()) - n_total
    partnered = int((nc > 1).sum())
    say(f"{2 * K} qubits, {n_total} samples ({partnered} with a partner, {n_hits} hits), "
        f"filter_bits {filter_bits or 'default'}")
    assert n_hits > 1000 and partnered > 1000
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    ham.set_tuning(strategy="enum", filter_bits=filter_bits)
    St = nqs.to_device_samples(S)
    la_t = torch.from_numpy(la).cuda()
    ph_t = torch.from_numpy(ph).cuda()
    G_dense, _, conn = W.closed_form_counts(K, K // 2)
    for precision, tol in (("fp64", TOL), ("fp32k", FP32_TOL)):
        e = ham.eloc(St, la_t, ph_t, precision=precision)
        ham.sync()
        r = torch.view_as_real(e).cpu().numpy()
        got = r[:, 0] + 1j * r[:, 1]
        st = ham.stats()
        plan = ham.plan()
        say(f"{precision}: plan {plan}, stats {st}")
        assert plan["strategy"] == "enum" and plan["filter_partitions"] == 8
        assert st["enum_rounds"] > 0
        assert st["hits"] == n_hits
        G = ham.n_groups
        lo = n_total * (conn - (G_dense - G))
        assert lo <= st["probes"] <= n_total * conn
        _parity(got, ref, ab, tol)
        # the rows that have partners, separately (they carry the class routes)
        sel = nc > 1
        _parity(got[sel], ref[sel], ab[sel], tol)
        if precision == "fp32k":
            m_ref, _, _ = oracle.energy(np.ones(n_total, np.int64), ref)
            m32, _, _ = oracle.energy(np.ones(n_total, np.int64), got)
            say(f"fp32k |dRe E| = {abs(m32.real - m_ref.real):.3e} Ha")
            assert abs(m32.real - m_ref.real) <= ENERGY_TOL_HA
    ham.close()
