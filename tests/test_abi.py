"""The C-ABI library loads, exports every declared symbol and validates codes on
the host before touching the device (no GPU needed)."""
import ctypes

import numpy as np
import pytest

from paper_1008_4370_amd import decoder as d


def test_library_exports_every_header_symbol():
    L = d.lib()
    syms = d.header_symbols()
    assert {"ldpc_fd_create_code", "ldpc_fd_decode", "ldpc_fd_round", "ldpc_fd_destroy_code",
            "ldpc_fd_workspace_bytes", "ldpc_fd_code_info", "ldpc_fd_last_error"} <= set(syms)
    for s in syms:
        assert getattr(L, s) is not None


def _create(M, N, m, rp, col, val, poly=0):
    h = ctypes.c_void_p()
    rp = np.asarray(rp, np.int32)
    col = np.asarray(col, np.int32)
    val = np.asarray(val, np.uint16)
    rc = d.lib().ldpc_fd_create_code(M, N, m, rp.ctypes.data, col.ctypes.data, val.ctypes.data, poly,
                                     ctypes.byref(h))
    return rc, d.lib().ldpc_fd_last_error().decode()


@pytest.mark.parametrize("args,rc,msg", [
    ((1, 2, 1, [0, 2], [0, 1], [1, 1]), d.E_UNSUPPORTED, "m must"),
    ((1, 2, 9, [0, 2], [0, 1], [1, 1]), d.E_UNSUPPORTED, "m must"),
    ((1, 3, 2, [0, 2], [0, 1], [1, 1]), d.E_INVALID, "weight 0"),
    ((2, 2, 2, [0, 2, 4], [0, 1, 0, 1], [1, 4, 1, 1]), d.E_INVALID, "label"),
    ((2, 2, 2, [0, 2, 4], [0, 1, 0, 1], [1, 0, 1, 1]), d.E_INVALID, "label"),
    ((2, 2, 2, [0, 2, 4], [0, 0, 1, 1], [1, 1, 1, 1]), d.E_INVALID, "duplicate"),
    ((2, 2, 2, [0, 1, 4], [0, 0, 1, 1], [1, 1, 1, 1]), d.E_INVALID, "weight < 2"),
    ((2, 2, 2, [0, 2, 4], [0, 5, 0, 1], [1, 1, 1, 1]), d.E_INVALID, "out of range"),
    ((2, 2, 2, [1, 2, 4], [0, 1, 0, 1], [1, 1, 1, 1]), d.E_INVALID, "row_ptr"),
])
def test_create_code_rejects_bad_input(args, rc, msg):
    got, err = _create(*args)
    assert got == rc and msg in err


def test_create_code_rejects_non_primitive_polynomial():
    # x^4 + x^3 + x^2 + x + 1 is irreducible but not primitive (alpha has order 5)
    got, err = _create(2, 2, 4, [0, 2, 4], [0, 1, 0, 1], [1, 1, 1, 1], poly=0b11111)
    assert got == d.E_INVALID and "primitive" in err
    got, err = _create(2, 2, 4, [0, 2, 4], [0, 1, 0, 1], [1, 1, 1, 1], poly=0b1011)
    assert got == d.E_INVALID and "degree" in err


def test_row_weight_limit():
    """Rows heavier than 16 are rejected before any device allocation."""
    col = list(range(17)) * 2
    got, err = _create(2, 17, 5, [0, 17, 34], col, [1] * 34)
    assert got == d.E_UNSUPPORTED and "row weight" in err


def test_column_weight_limit():
    """Columns heavier than 16 are rejected before any device allocation; the
    column weights below that may be irregular."""
    rp = [2 * r for r in range(18)]
    col = [x for r in range(17) for x in (0, r + 1)]
    got, err = _create(17, 18, 3, rp, col, [1] * 34)
    assert got == d.E_UNSUPPORTED and "column weight" in err


def test_pool_submit_rejects_bad_llr_before_the_library_call():
    """Pool.submit checks type, shape, layout, device and tags before handing the
    pointer to ldpc_fd_pool_submit (which reads n * N * m floats from it)."""
    import types

    torch = pytest.importorskip("torch")
    pool = d.Pool.__new__(d.Pool)
    pool.codes = [types.SimpleNamespace(N=12, m=3)]
    pool.handle = None
    good = torch.zeros((4, 12, 3), dtype=torch.float32)
    bad = [
        (np.zeros((4, 12, 3), np.float32), "torch tensor"),
        (good.to(torch.float16), "float32"),
        (torch.zeros((4, 11, 3), dtype=torch.float32), "shape"),
        (torch.zeros((4, 12), dtype=torch.float32), "shape"),
        (torch.zeros((4, 3, 12), dtype=torch.float32).transpose(1, 2), "contiguous"),
        (good, "device memory"),   # a host tensor (this container has no GPU)
    ]
    for llr, msg in bad:
        with pytest.raises(ValueError, match=msg):
            pool.submit(0, llr, None, 10)
    with pytest.raises(ValueError, match="code index"):
        pool.submit(1, good, None, 10)
    pool.handle = None
