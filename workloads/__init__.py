"""Seeded synthetic inputs for the local-energy path.

This module is the one input producer shared by the CPU oracle and the GPU
library.  It draws molecule-shaped integrals, expands the second-quantised
Hamiltonian (Eq. 2) into Jordan-Wigner Pauli strings, draws unique
occupation-number samples from a fixed (N_alpha, N_beta) sector, integer
weights, log-amplitudes and phases.  It holds none of the local-energy
arithmetic (Eq. 5) and imports neither the oracle nor the GPU package.

Conventions
-----------
* Spin orbital (p, alpha) is qubit 2p, (p, beta) is qubit 2p+1 (ONV order of
  Sec. II-A).  Qubit j is bit j % 64 of word j // 64; a set bit is occupied.
* A Pauli term is (x, z, c) with P = i^{popc(x & z)} X^x Z^z, x and z packed
  as two uint64 words (lo word = qubits 0..63).
* Seeds: numpy PCG64 ``default_rng(prefix + [stream])`` with stream 0
  integrals, 1 samples, 2 weights, 3 log-amplitudes, 4 phases; each named
  workload has its own prefix, and Hamiltonian j of a batched family uses
  the prefix ``[seed, 100 + j]``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libjwgen.so")
_SRC_PATH = os.path.join(_HERE, "jw_expand.c")

DROP_THRESHOLD = 1e-12

# ---------------------------------------------------------------- packing


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """Pack a bool array [n, n_q] (n_q <= 128) into uint64 words [n, 2]."""
    bits = np.asarray(bits, dtype=bool)
    n, nq = bits.shape
    if nq > 128:
        raise ValueError("at most 128 qubits")
    full = np.zeros((n, 128), dtype=bool)
    full[:, :nq] = bits
    packed = np.packbits(full, axis=1, bitorder="little")  # [n, 16] uint8
    return np.ascontiguousarray(packed).view("<u8").reshape(n, 2).astype(np.uint64)


def unpack_bits(words: np.ndarray, nq: int) -> np.ndarray:
    """Inverse of pack_bits: uint64 [n, 2] -> bool [n, nq]."""
    w = np.ascontiguousarray(np.asarray(words, dtype="<u8").reshape(-1, 2))
    b = np.unpackbits(w.view(np.uint8).reshape(-1, 16), axis=1, bitorder="little")
    return b[:, :nq].astype(bool)


def spin_masks(nq: int) -> np.ndarray:
    """[2][2] uint64: alpha (even qubits) and beta (odd qubits) masks."""
    a = np.zeros((1, nq), dtype=bool)
    b = np.zeros((1, nq), dtype=bool)
    a[0, 0::2] = True
    b[0, 1::2] = True
    return np.concatenate([pack_bits(a), pack_bits(b)], axis=0)


# ---------------------------------------------------------------- integrals


def integrals(rng: np.random.Generator, K: int, L: float):
    """Seeded real integrals with the symmetries of real orbitals.

    h: upper triangle p <= q drawn N(0,1) in row-major order, scaled by
    exp(-|p-q|/L), mirrored.  (pq|rs): one N(0, 0.1) value per canonical
    quadruple (p >= q, r >= s, pq >= rs with pq = p(p+1)/2 + q), drawn in
    compound-index order, scaled by exp(-(|p-q| + |r-s|)/L) and copied to all
    eight permutations.
    """
    h = np.zeros((K, K))
    iu = np.triu_indices(K)
    vals = rng.normal(0.0, 1.0, size=iu[0].size)
    h[iu] = vals * np.exp(-np.abs(iu[0] - iu[1]) / L)
    h = h + np.triu(h, 1).T

    # compound pair index list in increasing order: pq = p(p+1)/2 + q, p >= q
    pairs = [(p, q) for p in range(K) for q in range(p + 1)]
    npair = len(pairs)
    pp = np.array([p for p, _ in pairs])
    qq = np.array([q for _, q in pairs])
    I, J = np.tril_indices(npair)  # I >= J, row-major = compound order
    v = rng.normal(0.0, 0.1, size=I.size)
    p, q, r, s = pp[I], qq[I], pp[J], qq[J]
    v = v * np.exp(-(np.abs(p - q) + np.abs(r - s)) / L)
    eri = np.zeros((K, K, K, K))
    for a, b, c, d in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                       (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
        eri[a, b, c, d] = v
    return h, eri


# ---------------------------------------------------------------- JW expansion


def _load_jw():
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH):
        build_jw()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.jw_build.restype = ctypes.c_void_p
    lib.jw_build.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                             ctypes.c_int, ctypes.c_int]
    lib.jw_count.restype = ctypes.c_int64
    lib.jw_count.argtypes = [ctypes.c_void_p]
    lib.jw_fetch.restype = None
    lib.jw_fetch.argtypes = [ctypes.c_void_p] * 5
    lib.jw_free.restype = None
    lib.jw_free.argtypes = [ctypes.c_void_p]
    return lib


def build_jw() -> str:
    """Compile the JW expansion helper with gcc (host code only)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
                           "-std=c11", _SRC_PATH, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_jw_lib = None


def jw_terms(h: np.ndarray, eri: np.ndarray, thresh: float = DROP_THRESHOLD,
             keep_odd: bool = False):
    """Jordan-Wigner Pauli terms of the spin-orbital Hamiltonian.

    Returns (x [T,2] u64, z [T,2] u64, c [T] f64), merged, with |c| < thresh
    dropped, sorted by (x_hi, x_lo, z_hi, z_lo).  With keep_odd the imaginary
    parts of odd-Y strings are returned too, as a fourth array.
    """
    global _jw_lib
    if _jw_lib is None:
        _jw_lib = _load_jw()
    K = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    n_parts = max(8, 2 * (os.cpu_count() or 8))
    res = _jw_lib.jw_build(K, h.ctypes.data, eri.ctypes.data, float(thresh), int(keep_odd),
                           n_parts)
    if not res:
        raise MemoryError("JW expansion failed")
    try:
        n = _jw_lib.jw_count(res)
        x = np.empty((n, 2), np.uint64)
        z = np.empty((n, 2), np.uint64)
        c = np.empty(n, np.float64)
        ci = np.empty(n, np.float64)
        _jw_lib.jw_fetch(res, x.ctypes.data, z.ctypes.data, c.ctypes.data, ci.ctypes.data)
    finally:
        _jw_lib.jw_free(res)
    if keep_odd:
        return x, z, c, ci
    return x, z, c


# ---------------------------------------------------------------- samples


def sector_states(K: int, na: int, nb: int) -> np.ndarray:
    """All bitstrings with na alpha and nb beta electrons, ascending integer order."""
    from itertools import combinations
    nq = 2 * K
    occ = []
    for a in combinations(range(K), na):
        for b in combinations(range(K), nb):
            bits = np.zeros(nq, dtype=bool)
            bits[[2 * i for i in a]] = True
            bits[[2 * i + 1 for i in b]] = True
            occ.append(bits)
    words = pack_bits(np.array(occ))
    order = np.lexsort((words[:, 0], words[:, 1]))
    return words[order]


def sector_samples(rng: np.random.Generator, K: int, na: int, nb: int, n_samples: int) -> np.ndarray:
    """Unique uniform draws from the (na, nb) sector, kept in draw order.

    Candidates are drawn in batches of n_samples: for each candidate the
    alpha occupied set is the first na columns of argsort(U[0,1)^K) and the
    beta set likewise from a second matrix; repeats of earlier draws are
    rejected until n_samples unique states are kept.
    """
    nq = 2 * K
    kept = []
    seen = set()
    total = 0
    while total < n_samples:
        ua = rng.random((n_samples, K))
        ub = rng.random((n_samples, K))
        oa = np.argsort(ua, axis=1, kind="stable")[:, :na]
        ob = np.argsort(ub, axis=1, kind="stable")[:, :nb]
        bits = np.zeros((n_samples, nq), dtype=bool)
        rows = np.arange(n_samples)[:, None]
        bits[rows, 2 * oa] = True
        bits[rows, 2 * ob + 1] = True
        words = pack_bits(bits)
        for w in words:
            key = (int(w[0]), int(w[1]))
            if key in seen:
                continue
            seen.add(key)
            kept.append(w)
            total += 1
            if total == n_samples:
                break
    return np.array(kept, dtype=np.uint64).reshape(n_samples, 2)


def planted_samples(rng: np.random.Generator, K: int, na: int, nb: int, n_base: int,
                    n_total: int, per_kind: int = 3) -> np.ndarray:
    """A uniform sector batch with planted neighbours (hit-heavy rows inside a
    hit-sparse batch).

    n_base uniform sector states each bring per_kind alpha singles, beta
    singles, alpha-alpha, beta-beta and alpha-beta doubles of themselves
    (occupied orbitals emptied, virtual ones filled, same spin counts); the
    rest of the batch is uniform sector draws.  Unique, shuffled, n_total
    states in all.
    """
    nq = 2 * K
    base = sector_samples(rng, K, na, nb, n_base)
    out = {}
    for w in base:
        out[(int(w[0]), int(w[1]))] = w
    bits = unpack_bits(base, nq)
    planted = []
    for row in bits:
        occ = [np.nonzero(row[s::2])[0] for s in (0, 1)]
        vir = [np.nonzero(~row[s::2])[0] for s in (0, 1)]
        kinds = ((1, 0), (0, 1), (2, 0), (0, 2), (1, 1))  # excitations per spin
        for ea, eb in kinds:
            for _ in range(per_kind):
                r = row.copy()
                ok = True
                for spin, e in ((0, ea), (1, eb)):
                    if e == 0:
                        continue
                    if len(occ[spin]) < e or len(vir[spin]) < e:
                        ok = False
                        break
                    i = rng.choice(occ[spin], e, replace=False)
                    a = rng.choice(vir[spin], e, replace=False)
                    r[2 * i + spin] = False
                    r[2 * a + spin] = True
                if ok:
                    planted.append(r)
    if planted:
        for w in pack_bits(np.array(planted)):
            out.setdefault((int(w[0]), int(w[1])), w)
    rest = n_total - len(out)
    if rest < 0:
        raise ValueError("n_total smaller than the planted set")
    extra = sector_samples(rng, K, na, nb, rest + len(out))
    for w in extra:
        if len(out) == n_total:
            break
        out.setdefault((int(w[0]), int(w[1])), w)
    if len(out) < n_total:
        raise ValueError("sector too small for n_total unique states")
    arr = np.array(list(out.values()), dtype=np.uint64).reshape(-1, 2)
    return arr[rng.permutation(arr.shape[0])]


def geometric_weights(rng: np.random.Generator, n: int) -> np.ndarray:
    """w = 1 + G with P(G = k) = 0.3 * 0.7^k (numpy's geometric(0.3), support >= 1)."""
    return rng.geometric(0.3, size=n).astype(np.int64)


# ---------------------------------------------------------------- workloads


@dataclass
class Workload:
    name: str
    n_qubits: int
    K: int
    n_alpha: int
    n_beta: int
    x: np.ndarray          # [T,2] u64
    z: np.ndarray          # [T,2] u64
    c: np.ndarray          # [T] f64
    spin_masks: np.ndarray  # [2,2] u64
    samples: np.ndarray    # [N,2] u64
    weights: np.ndarray    # [N] i64
    log_amp: np.ndarray    # [N] f64
    phase: np.ndarray      # [N] f64
    h: np.ndarray = field(repr=False, default=None)
    eri: np.ndarray = field(repr=False, default=None)

    @property
    def n_samples(self) -> int:
        return int(self.samples.shape[0])


_HAM_CACHE: dict = {}


def _hamiltonian(seed_prefix, K: int, L: float):
    key = (tuple(seed_prefix), K, L)
    if key not in _HAM_CACHE:
        _HAM_CACHE.clear()  # keep at most one (the 100-qubit table is ~400 MB)
        _HAM_CACHE[key] = _make_hamiltonian(seed_prefix, K, L)
    return _HAM_CACHE[key]


def _make_hamiltonian(seed_prefix, K: int, L: float):
    rng = np.random.default_rng(list(seed_prefix) + [0])
    h, eri = integrals(rng, K, L)
    x, z, c = jw_terms(h, eri)
    return h, eri, x, z, c


def molecule(seed_prefix, K: int, na: int, nb: int, n_samples: int, L: float = 4.0,
             log_sigma: float = 2.0, name: str = "", all_states: bool = False,
             unit_weights: bool = False) -> Workload:
    """One molecule-shaped workload drawn from the seed prefix."""
    seed_prefix = list(seed_prefix)
    h, eri, x, z, c = _hamiltonian(seed_prefix, K, L)
    if all_states:
        samples = sector_states(K, na, nb)
    else:
        samples = sector_samples(np.random.default_rng(seed_prefix + [1]), K, na, nb, n_samples)
    n = samples.shape[0]
    if unit_weights:
        w = np.ones(n, np.int64)
    else:
        w = geometric_weights(np.random.default_rng(seed_prefix + [2]), n)
    la = np.random.default_rng(seed_prefix + [3]).normal(0.0, log_sigma, size=n)
    ph = np.random.default_rng(seed_prefix + [4]).uniform(0.0, 2.0 * math.pi, size=n)
    return Workload(name=name, n_qubits=2 * K, K=K, n_alpha=na, n_beta=nb, x=x, z=z, c=c,
                    spin_masks=spin_masks(2 * K), samples=samples, weights=w, log_amp=la,
                    phase=ph, h=h, eri=eri)


WORKLOADS = ("nq12", "nq40", "nq100")


def workload(name: str, n_samples: int | None = None) -> Workload:
    """The named molecule-shaped workloads.

    nq12:  12 qubits (6 orbitals, 3a+3b), all 400 sector states, weight 1,
           log|psi| ~ N(0,1), phase ~ U[0, 2pi); seed prefix [0].
    nq40:  40 qubits (20 orbitals, 10a+10b), 65,536 unique samples,
           geometric weights, log|psi| ~ N(0,2); seed prefix [1].
    nq100: 100 qubits (50 orbitals, 25a+25b), decay length 6, 262,144
           samples; seed prefix [2].
    n_samples overrides the sample count (the same seeds, fewer draws),
    used for reduced test sizes.
    """
    if name == "nq12":
        return molecule([0], 6, 3, 3, 400, L=4.0, log_sigma=1.0, name="nq12-all400",
                        all_states=True, unit_weights=True)
    if name == "nq40":
        n = n_samples or 65536
        return molecule([1], 20, 10, 10, n, L=4.0, log_sigma=2.0, name=f"nq40-{n}")
    if name == "nq100":
        n = n_samples or 262144
        return molecule([2], 50, 25, 25, n, L=6.0, log_sigma=2.0, name=f"nq100-{n}")
    raise ValueError(f"unknown workload {name!r}; expected one of {WORKLOADS}")


def batched_family(j: int, seed: int = 3) -> Workload:
    """Hamiltonian j of the batched family: N_q drawn from {24, 28, ..., 80}
    at half filling, sample count log-uniform in [1e3, 2e5]; seed prefix
    [seed, 100 + j]."""
    rng = np.random.default_rng([seed, 100 + j, 5])
    nq = int(rng.choice(np.arange(24, 81, 4)))
    ns = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
    K = nq // 2
    n = K // 2
    sector = math.comb(K, n) ** 2
    ns = min(ns, sector // 2)
    return molecule([seed, 100 + j], K, n, K - n, ns, L=4.0, log_sigma=2.0,
                    name=f"family{seed}-{j}-nq{nq}-{ns}")


# ---------------------------------------------------------------- counting


def closed_form_counts(K: int, n: int):
    """Exact G, estimated T and in-sector connected states per sample for a
    dense molecular Hamiltonian with K spatial orbitals and n electrons per spin."""
    nq = 2 * K
    C = math.comb
    G = 1 + 2 * C(K, 2) + 2 * C(K, 4) + C(K, 2) ** 2
    T = (1 + nq + C(nq, 2)) + 4 * C(K, 2) * (nq - 1) + 12 * C(K, 4) + 4 * C(K, 2) ** 2
    conn = 2 * n * (K - n) + 2 * C(n, 2) * C(K - n, 2) + (n * (K - n)) ** 2
    return G, T, conn
