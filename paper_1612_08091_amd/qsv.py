"""ctypes binding of libqsv (include/qsv.h): argument marshalling only.

Every step of the simulation runs in the HIP library; this module converts
numpy arrays and Python sequences to the C ABI's pointers and sizes and turns
status codes into exceptions.  There is no fallback: if libqsv.so is missing
the import fails.  PyTorch is used only to hand the library a device stream
(and, optionally, a device buffer for the state).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsv.so")

C128, C64 = 0, 1
PERGATE, FUSED, TILED = 0, 1, 2
OP_MATRIX, OP_RX, OP_RY, OP_RZ = 0, 1, 2, 3
_DTYPES = {"c128": C128, "complex128": C128, C128: C128, "c64": C64, "complex64": C64, C64: C64}
_MODES = {"pergate": PERGATE, "fused": FUSED, "tiled": TILED, PERGATE: PERGATE, FUSED: FUSED,
          TILED: TILED}

STATUS = {0: "QSV_OK", 1: "QSV_EINVAL", 2: "QSV_ENOMEM", 3: "QSV_EDEVICE",
          4: "QSV_ENOTCLASSICAL", 5: "QSV_ESTATE", 6: "QSV_EUNSUPPORTED"}


class QsvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(code, str(code)), msg))
        self.code = code
        self.status = STATUS.get(code, str(code))


class NotClassicalError(QsvError):
    """Deallocation of a qubit in superposition (ProjectQ Sec. 4.1.1)."""


class Options(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int32), ("dtype", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("k_max", ctypes.c_int32), ("tile_bits", ctypes.c_int32),
                ("queue_limit", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("state", ctypes.c_void_p), ("state_bytes", ctypes.c_uint64),
                ("timing", ctypes.c_int32), ("reg_bits", ctypes.c_int32),
                ("relabel", ctypes.c_int32), ("mem_limit", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [("gates", ctypes.c_uint64), ("fused_ops", ctypes.c_uint64),
                ("passes", ctypes.c_uint64), ("kernels", ctypes.c_uint64),
                ("alg_bytes", ctypes.c_double), ("alg_flops", ctypes.c_double),
                ("amp_gate_updates", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class CircuitC(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("op", ctypes.c_void_p), ("k", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("qubits", ctypes.c_void_p), ("mat_off", ctypes.c_void_p),
                ("matrices", ctypes.c_void_p), ("param", ctypes.c_void_p),
                ("n_params", ctypes.c_int32), ("params", ctypes.c_void_p)]


class PauliSumC(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("xmask", ctypes.c_void_p),
                ("zmask", ctypes.c_void_p), ("coeff", ctypes.c_void_p)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("tile_bits", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("tune_cache", ctypes.c_char_p),
                ("big_per_workgroup", ctypes.c_int32)]


# name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "qsv_version": (ctypes.c_char_p, []),
    "qsv_last_error": (ctypes.c_char_p, [_P]),
    "qsv_options_default": (ctypes.c_int, [_P]),
    "qsv_create": (ctypes.c_int, [_P, _P]),
    "qsv_destroy": (ctypes.c_int, [_P]),
    "qsv_allocate": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "qsv_deallocate": (ctypes.c_int, [_P, ctypes.c_int32]),
    "qsv_qubits": (ctypes.c_int, [_P, _P, _P]),
    "qsv_apply": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P]),
    "qsv_apply_diag": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P]),
    "qsv_apply_math": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P]),
    "qsv_dm_apply": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P]),
    "qsv_dm_apply_kraus": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P]),
    "qsv_dm_probabilities": (ctypes.c_int, [_P, _P]),
    "qsv_dm_expectation": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "qsv_flush": (ctypes.c_int, [_P]),
    "qsv_synchronize": (ctypes.c_int, [_P]),
    "qsv_get_probability": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "qsv_get_probabilities": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "qsv_get_expectation": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "qsv_get_expectation_complex": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "qsv_measure": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "qsv_sample": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "qsv_apply_kraus_sampled": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P,
                                               ctypes.c_double, _P, _P]),
    "qsv_get_state": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "qsv_set_state": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "qsv_get_amplitudes": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P]),
    "qsv_state_pointer": (ctypes.c_int, [_P, _P, _P]),
    "qsv_get_stats": (ctypes.c_int, [_P, _P]),
    "qsv_reset": (ctypes.c_int, [_P]),
    "qsv_get_kernel_times": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "qsv_reset_stats": (ctypes.c_int, [_P]),
    "qsv_plan": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, _P, _P]),
    "qsv_check_tile_programs": (ctypes.c_int, [_P, _P, _P]),
    "qsv_copy_probe": (ctypes.c_int, [_P, _P, ctypes.c_uint64, _P]),
    "qsv_get_probability_noalloc": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.c_int32, _P, _P, _P, _P]),
    "qsv_adjoint_gradient": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "qsv_batch_create": (ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P]),
    "qsv_batch_run": (ctypes.c_int, [_P, _P]),
    "qsv_batch_info": (ctypes.c_int, [_P, _P, _P, _P]),
    "qsv_batch_destroy": (ctypes.c_int, [_P]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqsv.so is not built (run __graft_entry__.build() or "
                          "python paper_1612_08091_amd/build.py); there is no fallback path")
    # libqsv needs libamdhip64.so.7, the soname torch's bundled HIP runtime
    # also carries.  Loading torch first makes the dynamic loader bind libqsv
    # to that same runtime, so the process holds one HIP runtime and torch's
    # streams and buffers can be handed to the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _check(code: int, handle=None):
    if code != 0:
        msg = lib.qsv_last_error(handle)
        msg = msg.decode() if msg else ""
        if code == 4:
            raise NotClassicalError(code, msg)
        raise QsvError(code, msg)


def _torch_stream():
    """The current torch stream's handle if torch has a usable GPU, else None."""
    try:
        import torch
    except ImportError:
        return None
    if not torch.cuda.is_available():
        return None
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Simulator:
    """One state vector on the GPU (a libqsv handle).

    Qubit ids come from ``allocate``; gates are queued by ``apply`` and run on
    ``flush`` or on any call that reads the state (ProjectQ Sec. 4.3.2)."""

    def __init__(self, n_max: int = 30, dtype="c128", mode="tiled", k_max: int = 2,
                 tile_bits: int = 0, queue_limit: int = 0, stream=None, state=None,
                 use_torch_stream: bool = True, timing: bool = False, reg_bits: int = 0,
                 relabel: bool = True, mem_limit: int = 0):
        opt = Options()
        _check(lib.qsv_options_default(ctypes.byref(opt)))
        opt.n_max = n_max
        opt.dtype = _DTYPES[dtype]
        opt.mode = _MODES[mode]
        opt.k_max = k_max
        opt.tile_bits = tile_bits
        opt.queue_limit = queue_limit
        opt.timing = int(bool(timing))
        opt.reg_bits = reg_bits
        opt.relabel = int(bool(relabel))
        opt.mem_limit = int(mem_limit)
        if stream is None and use_torch_stream:
            stream = _torch_stream()
        opt.stream = stream
        self._state_ref = state
        if state is not None:          # a torch tensor on the device
            opt.state = ctypes.c_void_p(state.data_ptr())
            opt.state_bytes = state.numel() * state.element_size()
        self.dtype = opt.dtype
        self.np_dtype = np.complex128 if opt.dtype == C128 else np.complex64
        h = ctypes.c_void_p()
        _check(lib.qsv_create(ctypes.byref(opt), ctypes.byref(h)))
        self._h = h

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib.qsv_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- qubits ---------------------------------------------------------------
    def allocate(self, count: int = 1):
        ids = np.zeros(max(count, 1), dtype=np.int32)
        _check(lib.qsv_allocate(self._h, count, _ptr(ids)), self._h)
        return ids[:count].tolist()

    def deallocate(self, qid: int):
        _check(lib.qsv_deallocate(self._h, int(qid)), self._h)

    def qubits(self):
        n = ctypes.c_int32()
        _check(lib.qsv_qubits(self._h, ctypes.byref(n), None), self._h)
        ids = np.zeros(max(n.value, 1), dtype=np.int32)
        _check(lib.qsv_qubits(self._h, ctypes.byref(n), _ptr(ids)), self._h)
        return ids[: n.value].tolist()

    @property
    def n(self) -> int:
        return len(self.qubits())

    # -- gates ----------------------------------------------------------------
    def apply(self, matrix, targets: Sequence[int], controls: Sequence[int] = ()):
        u = np.ascontiguousarray(matrix, dtype=np.complex128)
        t = np.ascontiguousarray(list(targets) or [0], dtype=np.int32)
        c = np.ascontiguousarray(list(controls) or [0], dtype=np.int32)
        _check(lib.qsv_apply(self._h, _ptr(u), len(targets), _ptr(t), len(controls), _ptr(c)),
               self._h)

    def apply_diag(self, diag, targets: Sequence[int], controls: Sequence[int] = ()):
        """Queue diag(diag[0], ..., diag[2^k - 1]) on ``targets`` (bit j of the
        row index is targets[j]) under ``controls``."""
        d = np.ascontiguousarray(diag, dtype=np.complex128)
        t = np.ascontiguousarray(list(targets) or [0], dtype=np.int32)
        c = np.ascontiguousarray(list(controls) or [0], dtype=np.int32)
        if d.shape != (1 << len(targets),):
            raise ValueError("diag must have 2**len(targets) entries")
        _check(lib.qsv_apply_diag(self._h, _ptr(d), len(targets), _ptr(t), len(controls), _ptr(c)),
               self._h)

    def apply_math(self, qubits: Sequence[int], table, controls: Sequence[int] = ()):
        """Emulated math gate (Sec. 4.3.3): the register ``qubits`` (first =
        least significant bit) takes the value table[x]; ``table`` is a
        permutation of range(2**len(qubits)).  Flushes and runs at once."""
        tab = np.ascontiguousarray(table, dtype=np.uint32)
        if tab.shape != (1 << len(qubits),):
            raise ValueError("table must have 2**len(qubits) entries")
        q = np.ascontiguousarray(list(qubits) or [0], dtype=np.int32)
        c = np.ascontiguousarray(list(controls) or [0], dtype=np.int32)
        _check(lib.qsv_apply_math(self._h, len(qubits), _ptr(q), _ptr(tab), len(controls),
                                  _ptr(c)), self._h)

    def run(self, circuit, qubit_ids: Optional[Sequence[int]] = None):
        """Queue every gate of a circuit; circuit qubit j -> qubit_ids[j]."""
        ids = list(range(circuit.n)) if qubit_ids is None else list(qubit_ids)
        for g in circuit.gates:
            self.apply(g.matrix, [ids[q] for q in g.targets], [ids[q] for q in g.controls])

    def flush(self):
        _check(lib.qsv_flush(self._h), self._h)

    def synchronize(self):
        _check(lib.qsv_synchronize(self._h), self._h)

    # -- reductions -------------------------------------------------------------
    def get_probability(self, qubits: Sequence[int], bits: Sequence[int]) -> float:
        q = np.ascontiguousarray(list(qubits) or [0], dtype=np.int32)
        b = np.ascontiguousarray(list(bits) or [0], dtype=np.int8)
        out = ctypes.c_double()
        _check(lib.qsv_get_probability(self._h, len(qubits), _ptr(q), _ptr(b), ctypes.byref(out)),
               self._h)
        return out.value

    def norm2(self) -> float:
        return self.get_probability([], [])

    def get_probabilities(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.float64)
        _check(lib.qsv_get_probabilities(self._h, _ptr(out), 0), self._h)
        return out

    def get_probabilities_device(self, out_tensor):
        """Write the probabilities into a float64 torch tensor on the device."""
        _check(lib.qsv_get_probabilities(self._h, ctypes.c_void_p(out_tensor.data_ptr()), 1),
               self._h)
        return out_tensor

    def get_expectation(self, xmask, zmask, coeff) -> float:
        x = np.ascontiguousarray(xmask, dtype=np.uint64)
        z = np.ascontiguousarray(zmask, dtype=np.uint64)
        c = np.ascontiguousarray(coeff, dtype=np.float64)
        out = ctypes.c_double()
        _check(lib.qsv_get_expectation(self._h, len(c), _ptr(x), _ptr(z), _ptr(c),
                                       ctypes.byref(out)), self._h)
        return out.value

    def get_expectation_complex(self, xmask, zmask, coeff):
        """(Re, Im) of sum_t coeff[t] <P_t>; Im is zero up to rounding."""
        x = np.ascontiguousarray(xmask, dtype=np.uint64)
        z = np.ascontiguousarray(zmask, dtype=np.uint64)
        c = np.ascontiguousarray(coeff, dtype=np.float64)
        re, im = ctypes.c_double(), ctypes.c_double()
        _check(lib.qsv_get_expectation_complex(self._h, len(c), _ptr(x), _ptr(z), _ptr(c),
                                               ctypes.byref(re), ctypes.byref(im)), self._h)
        return re.value, im.value

    def expectation(self, ham, qubit_ids: Optional[Sequence[int]] = None) -> float:
        """<H> for a workloads.PauliSum whose bit j refers to qubit_ids[j]
        (default: qubit id j)."""
        if qubit_ids is None:
            return self.get_expectation(ham.xmask, ham.zmask, ham.coeff)
        ids = list(qubit_ids)

        def remap(m):
            out = 0
            for j, q in enumerate(ids):
                if (int(m) >> j) & 1:
                    out |= 1 << q
            return out
        x = np.array([remap(m) for m in ham.xmask.tolist()], dtype=np.uint64)
        z = np.array([remap(m) for m in ham.zmask.tolist()], dtype=np.uint64)
        return self.get_expectation(x, z, ham.coeff)

    def measure(self, qubits: Sequence[int], u: Sequence[float]):
        q = np.ascontiguousarray(list(qubits) or [0], dtype=np.int32)
        uu = np.ascontiguousarray(list(u) or [0.0], dtype=np.float64)
        out = np.zeros(max(len(qubits), 1), dtype=np.int8)
        _check(lib.qsv_measure(self._h, len(qubits), _ptr(q), _ptr(uu), _ptr(out)), self._h)
        return out[: len(qubits)].tolist()

    def apply_kraus_sampled(self, kraus, targets: Sequence[int], u: float):
        """One stochastic-trajectory step: replace the channel {K_j} on
        ``targets`` (k <= 2) by branch j, chosen with the uniform ``u`` from
        p_j = ||K_j psi||^2; the state becomes K_j psi / sqrt(p_j).  Returns
        (j, p) with p the array of branch probabilities."""
        ks = np.ascontiguousarray(np.stack([np.asarray(k, dtype=np.complex128) for k in kraus]))
        t = np.ascontiguousarray(list(targets), dtype=np.int32)
        chosen = ctypes.c_int32(-1)
        probs = np.zeros(len(ks), dtype=np.float64)
        _check(lib.qsv_apply_kraus_sampled(self._h, len(ks), _ptr(ks), len(t), _ptr(t), float(u),
                                           ctypes.byref(chosen), _ptr(probs)), self._h)
        return int(chosen.value), probs

    def sample(self, u) -> np.ndarray:
        uu = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros(max(len(uu), 1), dtype=np.uint64)
        _check(lib.qsv_sample(self._h, len(uu), _ptr(uu), _ptr(out)), self._h)
        return out[: len(uu)]

    def get_state(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=self.np_dtype)
        _check(lib.qsv_get_state(self._h, _ptr(out), 0), self._h)
        return out

    def set_state(self, psi: np.ndarray):
        a = np.ascontiguousarray(psi, dtype=self.np_dtype)
        if a.size != 1 << self.n:
            raise ValueError("state has %d amplitudes, expected %d" % (a.size, 1 << self.n))
        _check(lib.qsv_set_state(self._h, _ptr(a), 0), self._h)

    def get_amplitudes(self, indices) -> np.ndarray:
        idx = np.ascontiguousarray(indices, dtype=np.uint64)
        out = np.zeros(max(len(idx), 1), dtype=np.complex128)
        _check(lib.qsv_get_amplitudes(self._h, len(idx), _ptr(idx), _ptr(out)), self._h)
        return out[: len(idx)]

    def state_pointer(self):
        p, s = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib.qsv_state_pointer(self._h, ctypes.byref(p), ctypes.byref(s)), self._h)
        return p.value, s.value

    # -- introspection -----------------------------------------------------------
    def stats(self) -> dict:
        st = Stats()
        _check(lib.qsv_get_stats(self._h, ctypes.byref(st)), self._h)
        return st.as_dict()

    def reset_stats(self):
        _check(lib.qsv_reset_stats(self._h), self._h)

    def reset(self):
        """State back to |0...0> on the live qubits; queued gates dropped."""
        _check(lib.qsv_reset(self._h), self._h)

    KERNEL_CLASSES = {"tile": 0, "dense": 1, "mono": 2, "reduce": 3}

    def kernel_times(self) -> dict:
        """Per kernel class: (device ms, launches, algorithmic bytes), from HIP
        events (needs timing=True)."""
        out = {}
        for name, cls in self.KERNEL_CLASSES.items():
            ms, n, b = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_double()
            _check(lib.qsv_get_kernel_times(self._h, cls, ctypes.byref(ms), ctypes.byref(n),
                                            ctypes.byref(b)), self._h)
            out[name] = (ms.value, n.value, b.value)
        return out

    def plan(self, max_ops: int = 100000):
        """(operations, passes): operations as (matrix, targets, control mask)
        in execution order, planned from the queued gates (nothing runs)."""
        nops, npass = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.qsv_plan(self._h, ctypes.byref(nops), ctypes.byref(npass), 0, None, None,
                            None, None), self._h)
        m = min(nops.value, max_ops)
        ks = np.zeros(max(m, 1), dtype=np.int32)
        tg = np.zeros(max(m, 1) * 5, dtype=np.int32)
        cm = np.zeros(max(m, 1), dtype=np.uint64)
        mats = np.zeros(max(m, 1) * 2048, dtype=np.float64)
        _check(lib.qsv_plan(self._h, ctypes.byref(nops), ctypes.byref(npass), m, _ptr(ks),
                            _ptr(tg), _ptr(cm), _ptr(mats)), self._h)
        ops = []
        for i in range(m):
            k = int(ks[i])
            d = 1 << k
            mat = mats[i * 2048: i * 2048 + 2 * d * d].view(np.complex128).reshape(d, d).copy()
            ops.append((mat, tg[5 * i: 5 * i + k].tolist(), int(cm[i])))
        return ops, npass.value

    def check_tile_programs(self, state: np.ndarray):
        """Run the register-tile programs planned for the queued gates on a
        host copy of ``state`` (complex128, 2^n) through the library's host
        model of the kernel (qsv_check_tile_programs); returns (new state,
        counts).  ``state`` None: lower only, for the counts.  A test of the
        lowering; nothing runs on the device."""
        buf = None if state is None else np.ascontiguousarray(state, dtype=np.complex128).copy()
        info = np.zeros(10, dtype=np.int32)
        _check(lib.qsv_check_tile_programs(self._h, _ptr(buf), _ptr(info)), self._h)
        keys = ("passes", "reg_passes", "real_ops", "diag_ops", "remaps", "max_image",
                "instructions", "diag_merged", "local_remaps", "relabel_passes")
        return buf, dict(zip(keys, info.tolist()))


def copy_probe(src, dst, stream=None):
    """Enqueue the library's streaming copy of torch tensor ``src`` into
    ``dst`` (same byte size, device memory) on ``stream`` (default: torch's
    current stream); the caller times it."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy_probe: sizes differ")
    if stream is None:
        stream = _torch_stream()
    _check(lib.qsv_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                              nbytes, stream))


# ---------------------------------------------------------------------------
# flat circuits and Pauli sums for the adjoint and batched forms
# ---------------------------------------------------------------------------
_AXIS_OP = {"X": OP_RX, "Y": OP_RY, "Z": OP_RZ}


class FlatCircuit:
    """A workloads.Circuit as the flat arrays of qsv_circuit (kept alive here)."""

    def __init__(self, circuit, theta=None):
        gates = circuit.gates
        g = len(gates)
        self.op = np.zeros(max(g, 1), dtype=np.int32)
        self.k = np.zeros(max(g, 1), dtype=np.int32)
        self.c = np.zeros(max(g, 1), dtype=np.int32)
        self.qubits = np.zeros(max(g, 1) * 8, dtype=np.int32)
        self.mat_off = np.zeros(max(g, 1), dtype=np.int64)
        self.param = np.full(max(g, 1), -1, dtype=np.int32)
        mats = []
        off = 0
        for i, gt in enumerate(gates):
            qs = list(gt.targets) + list(gt.controls)
            self.k[i] = len(gt.targets)
            self.c[i] = len(gt.controls)
            self.qubits[8 * i: 8 * i + len(qs)] = qs
            if gt.param >= 0:
                self.op[i] = _AXIS_OP[gt.axis]
                self.param[i] = gt.param
            else:
                self.op[i] = OP_MATRIX
                self.mat_off[i] = off
                mats.append(np.ascontiguousarray(gt.matrix, dtype=np.complex128).ravel())
                off += gt.matrix.size
        self.matrices = (np.concatenate(mats) if mats else np.zeros(1, np.complex128)).view(
            np.float64).copy()
        th = circuit.theta if theta is None else theta
        self.params = np.ascontiguousarray(th if th is not None else np.zeros(1), dtype=np.float64)
        self.n_params = 0 if th is None else len(th)
        self.struct = CircuitC(circuit.n, g, _ptr(self.op).value, _ptr(self.k).value,
                               _ptr(self.c).value, _ptr(self.qubits).value,
                               _ptr(self.mat_off).value, _ptr(self.matrices).value,
                               _ptr(self.param).value, self.n_params, _ptr(self.params).value)

    def set_params(self, theta):
        self.params[:] = np.asarray(theta, dtype=np.float64)


class FlatPauli:
    def __init__(self, ham):
        self.x = np.ascontiguousarray(ham.xmask, dtype=np.uint64)
        self.z = np.ascontiguousarray(ham.zmask, dtype=np.uint64)
        self.c = np.ascontiguousarray(ham.coeff, dtype=np.float64)
        self.struct = PauliSumC(len(self.c), _ptr(self.x).value, _ptr(self.z).value,
                                _ptr(self.c).value)


def adjoint_gradient(sim: Simulator, circuit, ham, theta=None):
    """(<H>, d<H>/d theta) by adjoint differentiation in the library."""
    fc = FlatCircuit(circuit, theta)
    fp = FlatPauli(ham)
    val = ctypes.c_double()
    grad = np.zeros(max(fc.n_params, 1), dtype=np.float64)
    _check(lib.qsv_adjoint_gradient(sim._h, ctypes.byref(fc.struct), ctypes.byref(fp.struct),
                                    ctypes.byref(val), _ptr(grad)), sim._h)
    return val.value, grad[: fc.n_params]


class DensityMatrix:
    """An n-qubit density matrix on a handle of 2n qubits (vec(rho), row bits
    low, column bits high; see qsv_dm_apply).  Gates and Kraus channels queue
    and run through the fused tile passes like ordinary gates."""

    def __init__(self, n: int, dtype="c128", mode="tiled", k_max: int = 2, **kw):
        self.n = n
        self.sim = Simulator(n_max=2 * n, dtype=dtype, mode=mode, k_max=k_max, **kw)
        self.sim.allocate(2 * n)

    def close(self):
        self.sim.close()

    def apply(self, matrix, targets: Sequence[int], controls: Sequence[int] = ()):
        u = np.ascontiguousarray(matrix, dtype=np.complex128)
        t = np.ascontiguousarray(list(targets) or [0], dtype=np.int32)
        c = np.ascontiguousarray(list(controls) or [0], dtype=np.int32)
        _check(lib.qsv_dm_apply(self.sim._h, _ptr(u), len(targets), _ptr(t), len(controls),
                                _ptr(c)), self.sim._h)

    def channel(self, kraus, targets: Sequence[int]):
        ks = np.ascontiguousarray(np.stack([np.asarray(k, dtype=np.complex128) for k in kraus]))
        t = np.ascontiguousarray(list(targets), dtype=np.int32)
        _check(lib.qsv_dm_apply_kraus(self.sim._h, len(ks), _ptr(ks), len(targets), _ptr(t)),
               self.sim._h)

    def run(self, events):
        """Queue ("gate", U, targets, controls) / ("kraus", [K_j], targets) events."""
        for ev in events:
            if ev[0] == "gate":
                self.apply(ev[1], ev[2], ev[3])
            else:
                self.channel(ev[1], ev[2])

    def flush(self):
        self.sim.flush()

    def probabilities(self) -> np.ndarray:
        out = np.zeros(1 << self.n, dtype=np.float64)
        _check(lib.qsv_dm_probabilities(self.sim._h, _ptr(out)), self.sim._h)
        return out

    def expectation(self, ham) -> float:
        x = np.ascontiguousarray(ham.xmask, dtype=np.uint64)
        z = np.ascontiguousarray(ham.zmask, dtype=np.uint64)
        c = np.ascontiguousarray(ham.coeff, dtype=np.float64)
        out = ctypes.c_double()
        _check(lib.qsv_dm_expectation(self.sim._h, len(c), _ptr(x), _ptr(z), _ptr(c),
                                      ctypes.byref(out)), self.sim._h)
        return out.value

    def matrix(self) -> np.ndarray:
        """rho as a 2^n x 2^n array (host copy)."""
        v = self.sim.get_state()
        return v.reshape(1 << self.n, 1 << self.n).T.copy()


def math_table(func, widths: Sequence[int]) -> np.ndarray:
    """Tabulate a BasicMathGate-style function (Sec. 4.3.3) of several
    registers: ``func(*values) -> tuple of new values``, register r holding
    widths[r] bits, packed least significant register first.  ``func`` is
    called once on numpy arrays of all register values (so x + c, a * x % N
    and the like vectorise); the result must be a permutation."""
    total = int(sum(widths))
    x = np.arange(1 << total, dtype=np.uint64)
    vals, off = [], 0
    for w in widths:
        vals.append((x >> np.uint64(off)) & np.uint64((1 << w) - 1))
        off += w
    out = func(*vals)
    if not isinstance(out, (tuple, list)):
        out = (out,)
    packed, off = np.zeros_like(x), 0
    for w, v in zip(widths, out):
        packed |= (np.asarray(v, dtype=np.uint64) & np.uint64((1 << w) - 1)) << np.uint64(off)
        off += w
    return packed.astype(np.uint32)


class Batch:
    """Many small circuits with their Pauli sums, evaluated by one HIP-graph
    replay: circuits that fit in LDS in one persistent launch, larger ones
    pass-major (big_per_workgroup=True: each on one workgroup instead)."""

    def __init__(self, circuits, hams, dtype="c64", autotune=True, tile_bits=0,
                 use_graph=True, stream=None, tune_cache=None, big_per_workgroup=False):
        self._fc = [FlatCircuit(c) for c in circuits]
        self._fp = [FlatPauli(h) for h in hams]
        self.count = len(circuits)
        arr_c = (CircuitC * self.count)(*[f.struct for f in self._fc])
        arr_h = (PauliSumC * self.count)(*[f.struct for f in self._fp])
        self._arr = (arr_c, arr_h)
        if stream is None:
            stream = _torch_stream()
        self._cache = tune_cache.encode() if tune_cache else None
        opt = BatchOptions(_DTYPES[dtype], int(autotune), tile_bits, int(use_graph), stream,
                           self._cache, int(bool(big_per_workgroup)))
        h = ctypes.c_void_p()
        _check(lib.qsv_batch_create(self.count, arr_c, arr_h, ctypes.byref(opt), ctypes.byref(h)))
        self._h = h

    def run(self) -> np.ndarray:
        out = np.zeros(max(self.count, 1), dtype=np.float64)
        _check(lib.qsv_batch_run(self._h, _ptr(out)))
        return out[: self.count]

    def info(self):
        tb, kf, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib.qsv_batch_info(self._h, ctypes.byref(tb), ctypes.byref(kf), ctypes.byref(ms)))
        return {"tile_bits": tb.value, "k_fuse": kf.value, "last_ms": ms.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib.qsv_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
