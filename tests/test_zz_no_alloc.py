"""qsv_get_probability_noalloc, the entry point that allocates nothing,
against qsv_get_probability on the same states, through the C ABI.

Two calls in a row on one GPU share the library's static partial-sum array;
the second has a smaller state (fewer partial sums), so a stale value from the
first call would show.  Same kernels and the same grid as the existing entry
point, so the sums must agree to the last bit.
"""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

Q = None


def setup_module(module):
    global Q
    from paper_1612_08091_amd import qsv
    Q = qsv


def noalloc(state_ptr, dtype, n, positions, bits, out, stream):
    pos = np.ascontiguousarray(list(positions) or [0], dtype=np.int32)
    b = np.ascontiguousarray(list(bits) or [0], dtype=np.int8)
    code = Q.lib.qsv_get_probability_noalloc(
        ctypes.c_void_p(state_ptr), dtype, n, len(positions), Q._ptr(pos), Q._ptr(b),
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream))
    Q._check(code)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_probability_matches_existing_entry_point(dtype):
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    for n, seed in [(20, 11), (9, 12)]:            # second call: smaller state
        rng = np.random.default_rng(seed)
        circ = W.config0(n=n, layers=6, shots=1)[0]
        s = Q.Simulator(n_max=n, dtype=dtype, mode="tiled", use_torch_stream=False)
        ids = s.allocate(n)
        s.run(circ)
        s.flush()
        ptr, stream = s.state_pointer()
        cases = [([], []), ([ids[0]], [1]), ([ids[n - 1], ids[2]], [0, 1]),
                 (list(ids[:5]), rng.integers(0, 2, size=5).tolist())]
        for qs, bits in cases:
            want = s.get_probability(qs, bits)
            # qubit ids were allocated in order: id j sits at bit position j
            noalloc(ptr, s.dtype, n, qs, bits, out, stream)
            s.synchronize()
            torch.cuda.synchronize()
            got = float(out.cpu()[0])
            assert got == want, (n, dtype, qs, bits, got, want)
        s.close()


def test_noalloc_rejects_bad_arguments_without_device_work():
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    buf = torch.zeros(2 << 4, dtype=torch.float64, device="cuda")
    for n, pos, bits, dt in [(4, [4], [1], 0), (4, [1, 1], [0, 1], 0), (40, [], [], 0),
                             (4, [], [], 7)]:
        with pytest.raises(Q.QsvError) as ei:
            noalloc(buf.data_ptr(), dt, n, pos, bits, out, None)
        assert ei.value.code == 1
