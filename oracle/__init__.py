"""CPU FP64 oracle for the local-energy path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The GPU library
never calls it, and it shares no code with the GPU library (kernels, headers,
table builders or helpers).  Its only common dependency with the GPU side is
the seeded input producer in ``workloads``.

Contents
--------
* ``eloc``/``eloc_rows``: Eq. 5 over the sample set (sample-space energy,
  Sec. IV-C), by the literal double loop in ``eloc_oracle.c``.
* ``energy``: Eq. 1, the weighted mean of E_loc over unique samples with
  integer counts, and the weighted population variance, both two-pass with
  exactly rounded sums (``math.fsum``).
* ``dense``: independent brute-force checkers (Kronecker-product Pauli
  matrices, literal second-quantised operator algebra of Eq. 2 on bit
  strings, Slater-Condon rules).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eloc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build() -> str:
    """Compile the C oracle with gcc (OpenMP, no SIMD tuning beyond -O2)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC,
                           "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oracle_eloc.restype = ctypes.c_int
    lib.oracle_eloc.argtypes = [ctypes.c_int, I64, P, P, P, P, I64, P, P, P, P, P, P, ctypes.c_int]
    lib.oracle_eloc_rows.restype = ctypes.c_int
    lib.oracle_eloc_rows.argtypes = [ctypes.c_int, I64, P, P, P, P, I64, P, P, P, I64, P, P, P, P,
                                     ctypes.c_int]
    lib.oracle_pairs.restype = I64
    lib.oracle_pairs.argtypes = [I64, P, I64, P, P, I64]
    lib.oracle_hij.restype = None
    lib.oracle_hij.argtypes = [I64, P, P, P, P, P, P, P]
    lib.oracle_hij_batch.restype = ctypes.c_int
    lib.oracle_hij_batch.argtypes = [I64, P, P, P, P, I64, P, P, P]
    lib.oracle_n_groups.restype = I64
    lib.oracle_n_groups.argtypes = [I64, P]
    _lib = lib
    return lib


def _u64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(-1, 2))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data


def eloc(n_qubits, x, z, c, samples, log_amp, phase, c_im=None, threads=0):
    """E_loc(s_i) for every sample (Eq. 5 restricted to S).

    Returns (eloc complex128 [N], absum float64 [N], n_conn int64 [N]) where
    absum is sum over connected x' of |psi(x')/psi(x)| * sum_t |c_t| and
    n_conn counts the connected x' in S (x itself included).
    """
    lib = _load()
    x, z, s = _u64(x), _u64(z), _u64(samples)
    c = _f64(c)
    ci = None if c_im is None else _f64(c_im)
    la, ph = _f64(log_amp), _f64(phase)
    n = s.shape[0]
    out = np.zeros((n, 2))
    ab = np.zeros(n)
    nc = np.zeros(n, np.int64)
    rc = lib.oracle_eloc(int(n_qubits), x.shape[0], _ptr(x), _ptr(z), _ptr(c), _ptr(ci), n, _ptr(s),
                         _ptr(la), _ptr(ph), _ptr(out), _ptr(ab), _ptr(nc), int(threads))
    if rc != 0:
        raise MemoryError("oracle_eloc failed")
    return out[:, 0] + 1j * out[:, 1], ab, nc


def eloc_rows(n_qubits, x, z, c, samples, log_amp, phase, rows, c_im=None, threads=0):
    """E_loc for the samples listed in ``rows`` only (x' still over all of S)."""
    lib = _load()
    x, z, s = _u64(x), _u64(z), _u64(samples)
    c = _f64(c)
    ci = None if c_im is None else _f64(c_im)
    la, ph = _f64(log_amp), _f64(phase)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    m = rows.shape[0]
    out = np.zeros((m, 2))
    ab = np.zeros(m)
    nc = np.zeros(m, np.int64)
    rc = lib.oracle_eloc_rows(int(n_qubits), x.shape[0], _ptr(x), _ptr(z), _ptr(c), _ptr(ci),
                              s.shape[0], _ptr(s), _ptr(la), _ptr(ph), m, _ptr(rows), _ptr(out),
                              _ptr(ab), _ptr(nc), int(threads))
    if rc != 0:
        raise MemoryError("oracle_eloc_rows failed")
    return out[:, 0] + 1j * out[:, 1], ab, nc


def connected_pairs(x, samples):
    """All (i, j) with a term connecting s_i and s_j (x' = x included), row-major."""
    lib = _load()
    x, s = _u64(x), _u64(samples)
    n = lib.oracle_pairs(x.shape[0], _ptr(x), s.shape[0], _ptr(s), None, 0)
    out = np.zeros((max(n, 1), 2), np.int64)
    lib.oracle_pairs(x.shape[0], _ptr(x), s.shape[0], _ptr(s), _ptr(out), n)
    return out[:n]


def hij(x, z, c, bra, ket, c_im=None):
    """<bra|H|ket> for arrays of basis-state pairs ([n,2] u64 each)."""
    lib = _load()
    x, z = _u64(x), _u64(z)
    c = _f64(c)
    ci = None if c_im is None else _f64(c_im)
    bra, ket = _u64(bra), _u64(ket)
    out = np.zeros((bra.shape[0], 2))
    lib.oracle_hij_batch(x.shape[0], _ptr(x), _ptr(z), _ptr(c), _ptr(ci), bra.shape[0], _ptr(bra),
                         _ptr(ket), _ptr(out))
    return out[:, 0] + 1j * out[:, 1]


def n_groups(x):
    lib = _load()
    x = _u64(x)
    return int(lib.oracle_n_groups(x.shape[0], _ptr(x)))


def energy(weights, el):
    """Eq. 1 over unique samples with integer counts.

    Returns (mean complex, variance float, sum_w float): mean = sum w E / sum w,
    variance = sum w |E - mean|^2 / sum w (population form), two passes with
    exactly rounded sums.
    """
    w = np.asarray(weights, dtype=np.int64)
    el = np.asarray(el, dtype=np.complex128)
    sw = float(int(w.sum()))
    wf = w.astype(np.float64)
    mr = math.fsum((wf * el.real).tolist()) / sw
    mi = math.fsum((wf * el.imag).tolist()) / sw
    dev = (el.real - mr) ** 2 + (el.imag - mi) ** 2
    var = math.fsum((wf * dev).tolist()) / sw
    return complex(mr, mi), var, sw
