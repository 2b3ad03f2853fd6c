"""Host-side checks of libnqs.so that need no GPU: the library loads, exports
every entry point of include/nqs.h, and its table builder validates, folds,
merges and groups terms as documented."""
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_2506_23809_amd as nqs
import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "nqs.h")


def test_library_exports_every_declared_symbol():
    lib = nqs.load_library()
    text = open(HEADER).read()
    declared = set(re.findall(r"^\w[\w \*]*?\b(nqs_\w+)\s*\(", text, flags=re.M))
    assert declared == set(nqs.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.nqs_version() == 101


def _ny(x, z):
    return np.array([bin(int(a) & int(b)).count("1") + bin(int(a2) & int(b2)).count("1")
                     for (a, a2), (b, b2) in zip(x, z)])


@pytest.mark.parametrize("name", ["nq12", "nq40"])
def test_table_groups_and_folds(name, workload_cache):
    w = workload_cache(("workload", name))
    gx, go, tz, tc = nqs.table_host(w.n_qubits, w.x, w.z, w.c)
    G, T, _ = W.closed_form_counts(w.K, w.n_alpha)
    assert gx.shape[0] == G == oracle.n_groups(w.x)
    assert tz.shape[0] == T
    # group 0 is the diagonal; groups ascend by (hi, lo)
    assert gx[0, 0] == 0 and gx[0, 1] == 0
    key = gx[:, 1].astype(object) * (1 << 64) + gx[:, 0].astype(object)
    assert all(key[k] < key[k + 1] for k in range(len(key) - 1))
    assert go[0] == 0 and go[-1] == T and np.all(np.diff(go) > 0)
    # the input list is already merged and sorted, so terms map one to one;
    # each coefficient is c * (-1)^{ny/2}
    tx = np.repeat(gx, np.diff(go), axis=0)
    assert np.array_equal(tx, w.x) and np.array_equal(tz, w.z)
    sign = np.where((_ny(w.x, w.z) // 2) % 2 == 1, -1.0, 1.0)
    assert np.array_equal(tc, w.c * sign)


def test_table_merges_equal_strings_in_input_order():
    x = np.array([[3, 0], [0, 0], [3, 0], [3, 0], [1, 0]], np.uint64)
    z = np.array([[0, 0], [2, 0], [0, 0], [3, 0], [0, 0]], np.uint64)
    c = np.array([0.5, 1.0, 0.25, -2.0, 3.0])
    gx, go, tz, tc = nqs.table_host(4, x, z, c)
    assert gx.tolist() == [[0, 0], [1, 0], [3, 0]]
    assert go.tolist() == [0, 1, 2, 4]
    assert tz.tolist() == [[2, 0], [0, 0], [0, 0], [3, 0]]
    # (X=3, Z=0) merged 0.5 + 0.25; (X=3, Z=3) has two Y factors: -(-2.0)
    assert tc.tolist() == [1.0, 3.0, 0.75, 2.0]


def test_table_rejections():
    ok_x = np.array([[1, 0]], np.uint64)
    ok_z = np.array([[0, 0]], np.uint64)
    with pytest.raises(nqs.NQSError) as e:
        nqs.table_host(4, np.array([[1, 0]], np.uint64), np.array([[1, 0]], np.uint64), [1.0])
    assert e.value.code == nqs.NQS_E_NONREAL
    with pytest.raises(nqs.NQSError) as e:
        nqs.table_host(4, np.array([[1 << 4, 0]], np.uint64), ok_z, [1.0])
    assert e.value.code == nqs.NQS_E_RANGE
    with pytest.raises(nqs.NQSError) as e:
        nqs.table_host(64, ok_x, np.array([[0, 1]], np.uint64), [1.0])
    assert e.value.code == nqs.NQS_E_RANGE
    for bad_nq in (0, 128, -3):
        with pytest.raises(nqs.NQSError) as e:
            nqs.table_host(bad_nq, ok_x, ok_z, [1.0])
        assert e.value.code == nqs.NQS_E_RANGE
    for bad_c in (math.nan, math.inf):
        with pytest.raises(nqs.NQSError) as e:
            nqs.table_host(4, ok_x, ok_z, [bad_c])
        assert e.value.code == nqs.NQS_E_ARG
    # 127 qubits: top bit allowed
    gx, go, tz, tc = nqs.table_host(127, np.array([[0, 1 << 62]], np.uint64), ok_z, [2.0])
    assert gx.tolist() == [[0, 1 << 62]] and tc.tolist() == [2.0]
    # Y on two qubits: ny = 2 folds the sign
    gx, go, tz, tc = nqs.table_host(4, np.array([[3, 0]], np.uint64), np.array([[3, 0]], np.uint64),
                                    [0.75])
    assert tc.tolist() == [-0.75]
    # empty table
    gx, go, tz, tc = nqs.table_host(4, np.zeros((0, 2), np.uint64), np.zeros((0, 2), np.uint64), [])
    assert gx.shape[0] == 0 and go.tolist() == [0] and tz.shape[0] == 0
    lib_ = nqs.load_library()
    G = __import__("ctypes").c_int64()
    rc = lib_.nqs_table_host(4, 1, None, None, None, __import__("ctypes").byref(G),
                             __import__("ctypes").byref(G), None, None, None, None)
    assert rc == nqs.NQS_E_ARG


def test_api_argument_errors_without_device():
    """Calls that fail on their arguments return codes before touching a device."""
    import ctypes
    lib = nqs.load_library()
    assert lib.nqs_ham_create(None, 4, 0, None, None, None, None, None) == nqs.NQS_E_ARG
    assert lib.nqs_eloc_eval(None, 1, None, None, None, None, None, 0, None) == nqs.NQS_E_STATE
    assert lib.nqs_sync(None, None) == nqs.NQS_E_STATE
    assert lib.nqs_ham_info(None, None, None, None) == nqs.NQS_E_STATE
    assert lib.nqs_energy(0, None, None, None, None) == nqs.NQS_E_ARG
    assert lib.nqs_ham_destroy(None) == nqs.NQS_OK
    out = (ctypes.c_int64 * 6)()
    assert lib.nqs_eval_stats(None, out) == nqs.NQS_E_STATE
    h = ctypes.c_void_p()
    rc = lib.nqs_ham_create(ctypes.byref(h), 4, 1, np.array([1, 0], np.uint64).ctypes.data,
                            np.array([1, 0], np.uint64).ctypes.data,
                            np.array([1.0]).ctypes.data, None, None)
    assert rc == nqs.NQS_E_NONREAL and not h.value
    sm = np.array([[1, 0], [1, 0]], np.uint64)   # overlapping alpha / beta
    rc = lib.nqs_ham_create(ctypes.byref(h), 4, 1, np.array([3, 0], np.uint64).ctypes.data,
                            np.array([0, 0], np.uint64).ctypes.data,
                            np.array([1.0]).ctypes.data, sm.ctypes.data, None)
    assert rc == nqs.NQS_E_ARG
    assert b"overlap" in lib.nqs_last_error()
