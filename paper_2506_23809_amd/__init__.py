"""Python binding of libnqs.so, the MI355X local-energy library.

Argument marshalling only: every step of the local-energy path runs in the
library's HIP kernels.  PyTorch provides device memory and the current HIP
stream.  There is no CPU fallback: if ``libnqs.so`` is missing the import of
the library raises.

    ham = Hamiltonian(x, z, c, n_qubits, spin_masks)      # nqs_ham_create
    e   = ham.eloc(samples, log_amp, phase, weights)        # nqs_eloc_eval -> complex128 [n]
    mean, var, sum_w = energy(weights, e)                   # nqs_energy
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# NQS_LIBRARY names another build of the library (the host-only sanitizer
# build of the table builder, which exports only its host entry points)
LIB_PATH = os.environ.get("NQS_LIBRARY") or os.path.join(_HERE, "libnqs.so")

NQS_OK = 0
NQS_E_ARG = -1
NQS_E_RANGE = -2
NQS_E_NONREAL = -3
NQS_E_DUPLICATE = -4
NQS_E_NOMEM = -5
NQS_E_DEVICE = -6
NQS_E_STATE = -7

NQS_FP64 = 0
NQS_FP32_KAHAN = 1
NOALLOC_SCRATCH_BYTES = 160 << 20  # NQS_NOALLOC_SCRATCH_BYTES
_PRECISION = {"fp64": NQS_FP64, "fp32k": NQS_FP32_KAHAN, "fp32_kahan": NQS_FP32_KAHAN}

# Every symbol include/nqs.h declares.
EXPORTS = ("nqs_last_error", "nqs_version", "nqs_ham_create", "nqs_ham_create_integrals",
           "nqs_ham_info", "nqs_ham_destroy",
           "nqs_table_host", "nqs_diag_tiles_host", "nqs_eloc_eval", "nqs_energy",
           "nqs_eloc_energy", "nqs_sync", "nqs_eval_stats",
           "nqs_eval_plan", "nqs_debug_fail_allocs", "nqs_eloc_eval_noalloc",
           "nqs_debug_dump", "nqs_profile", "nqs_last_kernel_ms", "nqs_last_stage_ms", "nqs_set_tuning",
           "nqs_get_tuning", "nqs_autotune", "nqs_batch_create", "nqs_batch_launch",
           "nqs_batch_capture", "nqs_batch_replay", "nqs_batch_destroy", "nqs_server_create",
           "nqs_server_add_ham", "nqs_server_submit", "nqs_server_poll", "nqs_server_drain",
           "nqs_server_stats", "nqs_server_destroy")


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


STRATEGIES = {"auto": 0, "stream": 1, "enum": 2, "join": 3}
STRATEGY_NAMES = {v: k for k, v in STRATEGIES.items()}


class Tuning(ctypes.Structure):
    """nqs_tuning: streaming block size, filter bits per sample, work items per CU,
    lookup strategy (0 auto, 1 streaming, 2 enumeration, 3 pair join)."""
    _fields_ = [("threads", ctypes.c_int32), ("filter_bits", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("strategy", ctypes.c_int32)]

    def as_dict(self):
        return {"threads": self.threads, "filter_bits": self.filter_bits,
                "blocks_per_cu": self.blocks_per_cu,
                "strategy": STRATEGY_NAMES.get(self.strategy, self.strategy)}


class BatchItem(ctypes.Structure):
    _fields_ = [("ham", ctypes.c_void_p), ("n", ctypes.c_int64), ("samples", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("log_amp", ctypes.c_void_p),
                ("phase", ctypes.c_void_p), ("eloc", ctypes.c_void_p)]


class NQSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nqs error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libnqs.so and declare its signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2506_23809_amd/build.py "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(path)
    P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    sig = {
        "nqs_last_error": (ctypes.c_char_p, []),
        "nqs_version": (I, []),
        "nqs_ham_create": (I, [P, I, I64, P, P, P, P, P]),
        "nqs_ham_create_integrals": (I, [P, I, P, P, P]),
        "nqs_ham_info": (I, [P, P, P, P]),
        "nqs_ham_destroy": (I, [P]),
        "nqs_table_host": (I, [I, I64, P, P, P, P, P, P, P, P, P]),
        "nqs_diag_tiles_host": (I, [I, I64, P, P, P, P, P, P, P, P]),
        "nqs_eloc_eval": (I, [P, I64, P, P, P, P, P, I, P]),
        "nqs_eloc_eval_noalloc": (I, [P, I64, P, P, P, P, P, I, P]),
        "nqs_energy": (I, [I64, P, P, P, P]),
        "nqs_eloc_energy": (I, [P, I64, P, P, P, P, P, I, P, P]),
        "nqs_sync": (I, [P, P]),
        "nqs_eval_stats": (I, [P, P]),
        "nqs_eval_plan": (I, [P, P]),
        "nqs_debug_fail_allocs": (I, [I]),
        "nqs_debug_dump": (I, [P, I64, P, P, P, P, P, P, P]),
        "nqs_profile": (I, [P, I]),
        "nqs_last_kernel_ms": (I, [P, P]),
        "nqs_last_stage_ms": (I, [P, P]),
        "nqs_set_tuning": (I, [P, P]),
        "nqs_get_tuning": (I, [P, P]),
        "nqs_autotune": (I, [P, I64, P, P, P, P, I, ctypes.c_char_p, P, P, P]),
        "nqs_batch_create": (I, [P, I, P, I, I, P]),
        "nqs_batch_launch": (I, [P, P]),
        "nqs_batch_capture": (I, [P, P]),
        "nqs_batch_replay": (I, [P, P]),
        "nqs_batch_destroy": (I, [P]),
        "nqs_server_create": (I, [P, P]),
        "nqs_server_add_ham": (I, [P, P, I64]),
        "nqs_server_submit": (I, [P, P, P]),
        "nqs_server_poll": (I, [P, P, P, I, P]),
        "nqs_server_drain": (I, [P, ctypes.c_double]),
        "nqs_server_stats": (I, [P, P]),
        "nqs_server_destroy": (I, [P]),
    }
    for name, (res, args) in sig.items():
        # a host-only build lacks the device entry points: those stay unbound
        # (calling one raises AttributeError); the export test checks that
        # the full library has every one
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != NQS_OK:
        raise NQSError(rc, load_library().nqs_last_error().decode())


def _np_u64(a, shape_cols=2):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(-1, shape_cols))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, dtype, ncols=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if ncols is not None and (t.dim() != 2 or t.shape[1] != ncols):
        raise ValueError(f"expected shape [n, {ncols}]")
    return ctypes.c_void_p(t.data_ptr())


def table_host(n_qubits, x, z, c):
    """Host-only table builder (nqs_table_host): (group_x, group_off, term_z, term_c)."""
    lib = load_library()
    x, z = _np_u64(x), _np_u64(z)
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    G = ctypes.c_int64()
    T = ctypes.c_int64()
    args = (int(n_qubits), x.shape[0], x.ctypes.data, z.ctypes.data, c.ctypes.data)
    _check(lib.nqs_table_host(*args, ctypes.byref(G), ctypes.byref(T), None, None, None, None))
    gx = np.zeros((G.value, 2), np.uint64)
    go = np.zeros(G.value + 1, np.int64)
    tz = np.zeros((T.value, 2), np.uint64)
    tc = np.zeros(T.value, np.float64)
    _check(lib.nqs_table_host(*args, ctypes.byref(G), ctypes.byref(T), gx.ctypes.data,
                              go.ctypes.data, tz.ctypes.data, tc.ctypes.data))
    return gx, go, tz, tc


def diag_tiles_host(n_qubits, x, z, c, spin_masks=None):
    """Host-only digit tiles of the occupation-form diagonal
    (nqs_diag_tiles_host): (tiles int8 array, d0, scale); tiles is empty when
    the table has no occupation form."""
    lib = load_library()
    x, z = _np_u64(x), _np_u64(z)
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    sm = None if spin_masks is None else _np_u64(spin_masks)
    nb = ctypes.c_int64()
    d0 = ctypes.c_double()
    sc = ctypes.c_double()
    args = (int(n_qubits), x.shape[0], x.ctypes.data, z.ctypes.data, c.ctypes.data,
            None if sm is None else sm.ctypes.data)
    _check(lib.nqs_diag_tiles_host(*args, ctypes.byref(nb), None, None, None))
    tiles = np.zeros(nb.value, np.int8)
    _check(lib.nqs_diag_tiles_host(*args, ctypes.byref(nb), tiles.ctypes.data if nb.value else None,
                                   ctypes.byref(d0), ctypes.byref(sc)))
    return tiles, d0.value, sc.value


class Hamiltonian:
    """A resident Pauli table on the current device (nqs_ham_create)."""

    def __init__(self, x, z, c, n_qubits, spin_masks=None, stream=None):
        lib = load_library()
        x, z = _np_u64(x), _np_u64(z)
        c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        if not (x.shape[0] == z.shape[0] == c.shape[0]):
            raise ValueError("x, z and c must have the same number of terms")
        sm = None if spin_masks is None else _np_u64(spin_masks)
        h = ctypes.c_void_p()
        _check(lib.nqs_ham_create(ctypes.byref(h), int(n_qubits), x.shape[0], x.ctypes.data,
                                  z.ctypes.data, c.ctypes.data,
                                  None if sm is None else sm.ctypes.data, _stream(stream)))
        self._h = h
        self.n_qubits = int(n_qubits)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().nqs_ham_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @classmethod
    def from_integrals(cls, h1e, eri, stream=None):
        """nqs_ham_create_integrals: the Slater-Condon form from h_pq and (pq|rs)."""
        lib = load_library()
        h1e = np.ascontiguousarray(np.asarray(h1e, dtype=np.float64))
        eri = np.ascontiguousarray(np.asarray(eri, dtype=np.float64))
        K = h1e.shape[0]
        if h1e.shape != (K, K) or eri.shape != (K, K, K, K):
            raise ValueError("h1e must be [K, K] and eri [K, K, K, K]")
        h = ctypes.c_void_p()
        _check(lib.nqs_ham_create_integrals(ctypes.byref(h), K, h1e.ctypes.data, eri.ctypes.data,
                                            _stream(stream)))
        self = cls.__new__(cls)
        self._h = h
        self.n_qubits = 2 * K
        return self

    @property
    def handle(self):
        return self._h

    def info(self):
        G, T, B = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().nqs_ham_info(self._h, ctypes.byref(G), ctypes.byref(T),
                                           ctypes.byref(B)))
        return G.value, T.value, B.value

    @property
    def n_groups(self):
        return self.info()[0]

    @property
    def n_terms(self):
        return self.info()[1]

    def eloc_into(self, out, samples, log_amp, phase, weights=None, precision="fp64",
                  stream=None):
        """nqs_eloc_eval into a float64 [n, 2] device tensor (asynchronous)."""
        import torch
        n = samples.shape[0]
        wp = None if weights is None else _dptr(weights, torch.int64)
        _check(load_library().nqs_eloc_eval(
            self._h, n, _dptr(samples, torch.int64, 2), wp, _dptr(log_amp, torch.float64),
            _dptr(phase, torch.float64), _dptr(out, torch.float64, 2), _PRECISION[precision],
            _stream(stream)))
        return out

    def eloc_noalloc_into(self, out, samples, log_amp, phase, weights=None, precision="fp64",
                          stream=None):
        """nqs_eloc_eval_noalloc: as eloc_into, with the library's fixed
        scratch array instead of allocated scratch (calls on one device must
        not overlap)."""
        import torch
        n = samples.shape[0]
        wp = None if weights is None else _dptr(weights, torch.int64)
        _check(load_library().nqs_eloc_eval_noalloc(
            self._h, n, _dptr(samples, torch.int64, 2), wp, _dptr(log_amp, torch.float64),
            _dptr(phase, torch.float64), _dptr(out, torch.float64, 2), _PRECISION[precision],
            _stream(stream)))
        return out

    def eloc_energy_into(self, out, samples, log_amp, phase, weights, precision="fp64",
                         stream=None):
        """nqs_eloc_energy: E_loc into out (float64 [n, 2]) and Eq. 1 over it
        in one launch sequence; returns (mean complex, variance, sum_w) and
        synchronises the stream."""
        import torch
        n = samples.shape[0]
        res = (ctypes.c_double * 4)()
        _check(load_library().nqs_eloc_energy(
            self._h, n, _dptr(samples, torch.int64, 2), _dptr(weights, torch.int64),
            _dptr(log_amp, torch.float64), _dptr(phase, torch.float64),
            _dptr(out, torch.float64, 2), _PRECISION[precision], res, _stream(stream)))
        return complex(res[0], res[1]), res[2], res[3]

    def eloc(self, samples, log_amp, phase, weights=None, precision="fp64", stream=None):
        """E_loc for a batch; returns a complex128 device tensor [n]."""
        import torch
        out = torch.empty((samples.shape[0], 2), dtype=torch.float64, device=samples.device)
        self.eloc_into(out, samples, log_amp, phase, weights, precision, stream)
        return torch.view_as_complex(out)

    def sync(self, stream=None):
        """Wait for the stream and raise the first device-detected error."""
        _check(load_library().nqs_sync(self._h, _stream(stream)))

    def stats(self):
        out = (ctypes.c_int64 * 6)()
        _check(load_library().nqs_eval_stats(self._h, out))
        return {"pairs": out[0], "probes": out[1], "hits": out[2], "terms": out[3],
                "candidates": out[4], "enum_rounds": out[5]}

    def plan(self):
        """nqs_eval_plan: the launch plan of the last evaluation."""
        out = (ctypes.c_int64 * 8)()
        _check(load_library().nqs_eval_plan(self._h, out))
        return {"strategy": STRATEGY_NAMES.get(out[0], out[0]), "filter_partitions": out[1],
                "partition_words": out[2], "stream_chunks": out[3], "n": out[4],
                "filter_words": out[5], "join_blocks": out[6], "join_ran": out[7]}

    def profile(self, enable=True):
        """Record HIP events around each kernel stage of later evaluations."""
        _check(load_library().nqs_profile(self._h, 1 if enable else 0))

    def last_kernel_ms(self):
        """(hash build, lookup kernel, finish kernel) durations of the last evaluation."""
        out = (ctypes.c_float * 3)()
        _check(load_library().nqs_last_kernel_ms(self._h, out))
        return tuple(out)

    def last_stage_ms(self):
        """nqs_last_stage_ms: (grouping, hash build, join pairs, lookup, finish,
        total) durations of the last evaluation, in ms."""
        out = (ctypes.c_float * 6)()
        _check(load_library().nqs_last_stage_ms(self._h, out))
        return tuple(out)

    def set_tuning(self, threads=0, filter_bits=0, blocks_per_cu=0, strategy="auto"):
        """nqs_set_tuning; all zeros (strategy "auto") restores the built-in plan.
        strategy: "auto", "stream", "enum" or "join"."""
        t = Tuning(threads, filter_bits, blocks_per_cu, STRATEGIES[strategy])
        _check(load_library().nqs_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        _check(load_library().nqs_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, samples, log_amp, phase, out=None, precision="fp64", cache_path=None,
                 stream=None):
        """nqs_autotune: returns (tuning dict, best ms or -1 when cached); out holds E_loc."""
        import torch
        n = samples.shape[0]
        if out is None:
            out = torch.empty((n, 2), dtype=torch.float64, device=samples.device)
        best = Tuning()
        ms = ctypes.c_double()
        cp = None if cache_path is None else str(cache_path).encode()
        _check(load_library().nqs_autotune(
            self._h, n, _dptr(samples, torch.int64, 2), _dptr(log_amp, torch.float64),
            _dptr(phase, torch.float64), _dptr(out, torch.float64, 2), _PRECISION[precision], cp,
            ctypes.byref(best), ctypes.byref(ms), _stream(stream)))
        return best.as_dict(), ms.value

    def debug_dump(self, samples, log_amp, phase, hit_idx=None, sign_bits=None, stream=None):
        """nqs_debug_dump: E_loc plus the recorded lookups / sign bits."""
        import torch
        n = samples.shape[0]
        out = torch.empty((n, 2), dtype=torch.float64, device=samples.device)
        hp = None if hit_idx is None else _dptr(hit_idx, torch.int32)
        sp = None if sign_bits is None else _dptr(sign_bits, torch.int32)
        _check(load_library().nqs_debug_dump(
            self._h, n, _dptr(samples, torch.int64, 2), _dptr(log_amp, torch.float64),
            _dptr(phase, torch.float64), _dptr(out, torch.float64, 2), hp, sp, _stream(stream)))
        return torch.view_as_complex(out)


class Batch:
    """nqs_batch_*: many (Hamiltonian, batch) jobs in one persistent launch.

    jobs: list of (Hamiltonian, samples, log_amp, phase, weights or None, out)
    with device tensors; out is float64 [n, 2].  The buffers are recorded:
    launch() and replay() read their current contents.
    """

    def __init__(self, jobs, precision="fp64", threads=0, stream=None):
        import torch
        arr = (BatchItem * len(jobs))()
        self._keep = []
        for k, (ham, S, la, ph, w, out) in enumerate(jobs):
            n = S.shape[0]
            arr[k].ham = ham.handle
            arr[k].n = n
            arr[k].samples = _dptr(S, torch.int64, 2).value if n else None
            arr[k].weights = None if w is None else _dptr(w, torch.int64).value
            arr[k].log_amp = _dptr(la, torch.float64).value if n else None
            arr[k].phase = _dptr(ph, torch.float64).value if n else None
            arr[k].eloc = _dptr(out, torch.float64, 2).value if n else None
            self._keep.append((ham, S, la, ph, w, out))
        b = ctypes.c_void_p()
        _check(load_library().nqs_batch_create(ctypes.byref(b), len(jobs), arr,
                                               _PRECISION[precision], int(threads),
                                               _stream(stream)))
        self._b = b

    def launch(self, stream=None):
        _check(load_library().nqs_batch_launch(self._b, _stream(stream)))

    def capture(self, stream):
        """Capture one evaluation into a HIP graph (stream must not be the default one)."""
        _check(load_library().nqs_batch_capture(self._b, _stream(stream)))

    def replay(self, stream=None):
        _check(load_library().nqs_batch_replay(self._b, _stream(stream)))

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            _check(load_library().nqs_batch_destroy(self._b))
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _item(ham, S, la, ph, w, out):
    import torch
    n = S.shape[0]
    it = BatchItem()
    it.ham = ham.handle
    it.n = n
    it.samples = _dptr(S, torch.int64, 2).value if n else None
    it.weights = None if w is None else _dptr(w, torch.int64).value
    it.log_amp = _dptr(la, torch.float64).value if n else None
    it.phase = _dptr(ph, torch.float64).value if n else None
    it.eloc = _dptr(out, torch.float64, 2).value if n else None
    return it


class Server:
    """nqs_server_*: request loop with continuous batching over lanes (streams
    with their own scratch); see include/nqs.h."""

    def __init__(self, hbm_budget_bytes, streams=4, precision="fp64"):
        cfg = ServerConfig(int(hbm_budget_bytes), int(streams), _PRECISION[precision])
        s = ctypes.c_void_p()
        _check(load_library().nqs_server_create(ctypes.byref(s), ctypes.byref(cfg)))
        self._s = s
        self._keep = {}

    def add(self, ham, max_samples):
        _check(load_library().nqs_server_add_ham(self._s, ham.handle, int(max_samples)))

    def submit(self, ham, S, la, ph, w, out):
        """Enqueue one request; the tensors must stay alive until it finishes."""
        it = _item(ham, S, la, ph, w, out)
        t = ctypes.c_int64()
        _check(load_library().nqs_server_submit(self._s, ctypes.byref(it), ctypes.byref(t)))
        self._keep[t.value] = (S, la, ph, w, out)
        return t.value

    def poll(self, capacity=4096):
        tk = (ctypes.c_int64 * capacity)()
        lat = (ctypes.c_double * capacity)()
        n = ctypes.c_int()
        _check(load_library().nqs_server_poll(self._s, tk, lat, capacity, ctypes.byref(n)))
        out = [(tk[k], lat[k]) for k in range(n.value)]
        for t, _ in out:
            self._keep.pop(t, None)
        return out

    def drain(self, timeout_s=120.0):
        _check(load_library().nqs_server_drain(self._s, float(timeout_s)))

    def stats(self):
        o = (ctypes.c_int64 * 8)()
        _check(load_library().nqs_server_stats(self._s, o))
        keys = ("submitted", "completed", "rejected", "launches", "max_requests_in_flight",
                "max_launches_in_flight", "peak_bytes", "resident_bytes")
        return dict(zip(keys, list(o)))

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value:
            _check(load_library().nqs_server_destroy(self._s))
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_fail_allocs(k):
    """Test hook: the k-th scratch allocation from now fails once (0: off)."""
    _check(load_library().nqs_debug_fail_allocs(int(k)))


def energy(weights, eloc, stream=None):
    """nqs_energy: (mean complex, variance, sum_w); synchronises the stream."""
    import torch
    if eloc.dtype == torch.complex128:
        eloc = torch.view_as_real(eloc)
    out = (ctypes.c_double * 4)()
    n = weights.shape[0]
    _check(load_library().nqs_energy(n, _dptr(weights, torch.int64),
                                     _dptr(eloc.contiguous(), torch.float64, 2), out,
                                     _stream(stream)))
    return complex(out[0], out[1]), out[2], out[3]


def to_device_samples(words, device="cuda"):
    """uint64 [n, 2] numpy words -> int64 [n, 2] device tensor (same bits)."""
    import torch
    a = _np_u64(words).view(np.int64)
    return torch.from_numpy(a.copy()).to(device)
