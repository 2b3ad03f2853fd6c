"""The allocation-free entry point (nqs_eloc_eval_noalloc) against
nqs_eloc_eval, through the C ABI: the same kernels and plan on the library's
fixed scratch array, so the outputs must be identical bit for bit (and
within 1e-12 A(x) of the oracle).  Two calls in a row on the shared array,
the second with a smaller batch (it must not see the first call's hash);
then a batch too large for the array is refused before any launch."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import paper_2506_23809_amd as nqs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)
    sys.stdout.flush()


def _call(lib, fn, ham, S, la, ph, wt, out, precision):
    rc = getattr(lib, fn)(ham.handle, S.shape[0], ctypes.c_void_p(S.data_ptr()),
                          None if wt is None else ctypes.c_void_p(wt.data_ptr()),
                          ctypes.c_void_p(la.data_ptr()), ctypes.c_void_p(ph.data_ptr()),
                          ctypes.c_void_p(out.data_ptr()), precision, None)
    nqs._check(rc)


@pytest.mark.parametrize("name,sizes", [("nq40", (65536, 20000)), ("nq100", (262144, 3000)),
                                        ("nq12", (400, 57))])
def test_noalloc_equals_eloc_eval(name, sizes, workload_cache):
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    lib = nqs.load_library()
    w = workload_cache(("workload", name, sizes[0]) if name != "nq12" else ("workload", name))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    ref_ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    for precision in (nqs.NQS_FP64, nqs.NQS_FP32_KAHAN):
        for n in sizes:
            say(f"{w.name}: {n} samples, precision {precision}")
            S = nqs.to_device_samples(w.samples[:n])
            la = torch.from_numpy(w.log_amp[:n].copy()).cuda()
            ph = torch.from_numpy(w.phase[:n].copy()).cuda()
            wt = torch.from_numpy(w.weights[:n].copy()).cuda()
            a = torch.full((n, 2), float("nan"), dtype=torch.float64, device="cuda")
            b = torch.full((n, 2), float("nan"), dtype=torch.float64, device="cuda")
            _call(lib, "nqs_eloc_eval_noalloc", ham, S, la, ph, wt, a, precision)
            ham.sync()
            _call(lib, "nqs_eloc_eval", ref_ham, S, la, ph, wt, b, precision)
            ref_ham.sync()
            an, bn = a.cpu().numpy(), b.cpu().numpy()
            assert np.array_equal(an.view(np.uint64), bn.view(np.uint64))
            assert ham.stats()["hits"] == ref_ham.stats()["hits"]
            if precision == nqs.NQS_FP64:
                rows = np.unique(np.random.default_rng(n).choice(n, min(n, 64), replace=False))
                e_ref, ab, _ = oracle.eloc_rows(w.n_qubits, w.x, w.z, w.c, w.samples[:n],
                                                w.log_amp[:n], w.phase[:n], rows)
                got = an[rows, 0] + 1j * an[rows, 1]
                assert np.all(np.abs(got - e_ref) <= 1e-12 * ab)
    ham.close()
    ref_ham.close()


def test_noalloc_refuses_a_batch_larger_than_its_array(workload_cache):
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    lib = nqs.load_library()
    w = workload_cache(("workload", "nq12"))
    ham = nqs.Hamiltonian(w.x, w.z, w.c, w.n_qubits, w.spin_masks)
    # the size check comes before any pointer is used: a count far beyond
    # the array with small real buffers is refused on the host
    S = nqs.to_device_samples(w.samples)
    la = torch.zeros(400, dtype=torch.float64, device="cuda")
    out = torch.zeros((400, 2), dtype=torch.float64, device="cuda")
    say("noalloc: batch beyond the scratch array")
    rc = lib.nqs_eloc_eval_noalloc(ham.handle, 1 << 26, ctypes.c_void_p(S.data_ptr()), None,
                                   ctypes.c_void_p(la.data_ptr()), ctypes.c_void_p(la.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), 0, None)
    assert rc == nqs.NQS_E_ARG
    assert b"scratch" in lib.nqs_last_error()
    # the handle still works
    e = ham.eloc(S, la, la)
    ham.sync()
    assert e.shape[0] == 400
    ham.close()
