"""The C-ABI library loads, exports every symbol include/concpd.h declares,
and rejects invalid configurations on the host (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "concpd.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:concpd_status|const char\*)\s+(\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2302_05119_amd import _lib
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2302_05119_amd", "libconcpd.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, re.M))
    for s in syms:
        assert s in exported, s
        assert hasattr(lib, s)


def _cfg(S=2, R=5, L=(5, 0, 0), dims=None, tdt=1, cdt=1):
    from paper_2302_05119_amd._lib import Config
    dims = dims or [(10, 11, 12)] * S
    N = len(dims[0]) if dims else 3
    c = Config()
    c.order = N
    c.num_blocks = S
    c.rank = R
    for n in range(N):
        c.coupled[n] = L[n] if n < len(L) else 0
    arr = (ctypes.c_int64 * (N * S))(*[d for t in dims for d in t])
    c.dims = arr
    c.tensor_dtype = tdt
    c.compute_dtype = cdt
    c.update_core = 1
    c.restart = 1
    c.delta_w = 0.9999
    c.tol = 1e-8
    c.max_it = 100
    c.tucker_ranks = None
    c._keep = arr
    return c


def query(lib, c):
    n = ctypes.c_size_t()
    st = lib.concpd_query_workspace(ctypes.byref(c), ctypes.byref(n))
    return st, n.value


def test_query_workspace_valid(lib):
    st, n = query(lib, _cfg())
    assert st == 0 and n > 0
    st2, n2 = query(lib, _cfg(S=4))
    assert st2 == 0 and n2 > n


@pytest.mark.parametrize("kw,expect", [
    (dict(R=0), 1),
    (dict(R=65), 1),
    (dict(L=(6, 0, 0)), 1),
    (dict(dims=[(10, 11, 12), (9, 11, 12)]), 1),   # coupled mode with unequal sizes
    (dict(S=0), 1),
    (dict(tdt=1, cdt=0), 1),                        # F64 compute needs F64 tensors
    (dict(tdt=0, cdt=1), 2),                        # F64 tensors only with F64 compute
])
def test_invalid_configs_rejected_with_message(lib, kw, expect):
    st, _ = query(lib, _cfg(**kw))
    assert st == expect
    assert len(lib.concpd_last_error()) > 0


@pytest.mark.parametrize("ranks,expect", [((6, 3), 0), ((6, 6), 0), ((6, 2), 1), ((7, 6), 1), ((0, 6), 1)])
def test_block_ranks_validated(lib, ranks, expect):
    # R = 6 with L = (3, 0, 0): every R^(s) must lie in [3, 6]
    c = _cfg(S=2, R=6, L=(3, 0, 0))
    arr = (ctypes.c_int32 * 2)(*ranks)
    c.block_ranks = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
    st, _ = query(lib, c)
    assert st == expect, lib.concpd_last_error()


@pytest.mark.parametrize("masks,expect", [((0b11, 0, 0), 0), ((0b01, 0, 0), 0), ((0, 0, 0), 1), ((0b111, 0, 0), 1)])
def test_coupled_blocks_validated(lib, masks, expect):
    # S = 2, L = (3, 0, 0): a coupled mode needs a non-empty group of existing blocks
    c = _cfg(S=2, R=6, L=(3, 0, 0))
    arr = (ctypes.c_uint64 * 3)(*masks)
    c.coupled_blocks = ctypes.cast(arr, ctypes.POINTER(ctypes.c_uint64))
    st, _ = query(lib, c)
    assert st == expect, lib.concpd_last_error()


def test_coupled_blocks_allow_other_sizes_outside_the_group(lib):
    c = _cfg(S=2, R=6, L=(3, 0, 0), dims=[(10, 11, 12), (9, 11, 12)])
    st, _ = query(lib, c)
    assert st == 1                      # every block coupled: I_1 must agree
    arr = (ctypes.c_uint64 * 3)(0b01, 0, 0)
    c.coupled_blocks = ctypes.cast(arr, ctypes.POINTER(ctypes.c_uint64))
    st, _ = query(lib, c)
    assert st == 0, lib.concpd_last_error()


@pytest.mark.parametrize("order", [1, 2, 7])
def test_order_outside_three_to_six_rejected(lib, order):
    c = _cfg()
    c.order = order
    st, _ = query(lib, c)
    assert st == 1 and "order" in lib.concpd_last_error().decode()


def test_order_four_to_six_accepted_with_f32_or_f64(lib):
    # the N-way model of Section II-C: dims[N s + n], L_n per mode
    for N in (4, 5, 6):
        dims = [tuple(6 + n for n in range(N))] * 3
        st, n4 = query(lib, _cfg(S=3, R=4, L=(2,) * N, dims=dims))
        assert st == 0, lib.concpd_last_error()
        st, n8 = query(lib, _cfg(S=3, R=4, L=(2,) * N, dims=dims, tdt=0, cdt=0))
        assert st == 0 and n8 > n4
    # a bigger last mode needs more workspace
    st_a, a = query(lib, _cfg(S=2, R=4, L=(0, 0, 0, 0), dims=[(5, 6, 7, 8)] * 2))
    st_b, b = query(lib, _cfg(S=2, R=4, L=(0, 0, 0, 0), dims=[(5, 6, 7, 80)] * 2))
    assert st_a == 0 and st_b == 0 and b > a


@pytest.mark.parametrize("kw,expect", [
    (dict(cdt=2), 2),                                              # BF16 compute: order 3 only
    (dict(cdt=3), 2),                                              # FP16 compute: order 3 only
    (dict(L=(0, 0, 0, 3), dims=[(5, 6, 7, 8), (5, 6, 7, 9)]), 1),  # coupled mode 4 with unequal sizes
    (dict(L=(0, 0, 0, 6)), 1),                                     # L_4 > R
])
def test_order_four_invalid_or_unsupported(lib, kw, expect):
    base = dict(S=2, R=5, L=(0, 0, 0, 0), dims=[(5, 6, 7, 8)] * 2)
    base.update(kw)
    st, _ = query(lib, _cfg(**base))
    assert st == expect, lib.concpd_last_error()


def test_order_four_rejects_tucker_ranks(lib):
    c = _cfg(S=1, R=4, L=(0, 0, 0, 0), dims=[(5, 6, 7, 8)])
    tr = (ctypes.c_int32 * 4)(2, 2, 2, 2)
    c.tucker_ranks = ctypes.cast(tr, ctypes.POINTER(ctypes.c_int32))
    st, _ = query(lib, c)
    assert st == 2 and "order 3" in lib.concpd_last_error().decode()


def test_init_rejects_null_arguments_without_device(lib):
    c = _cfg()
    ctx = ctypes.c_void_p()
    st = lib.concpd_init(ctypes.byref(c), None, None, None, 0, None, 0, None, ctypes.byref(ctx))
    assert st == 1 and not ctx.value


def test_calls_on_null_context_fail_cleanly(lib):
    from paper_2302_05119_amd._lib import Stats
    assert lib.concpd_step(None, 1, ctypes.byref(Stats())) == 1
    assert lib.lra_step(None, 1, None) == 1
    assert lib.concpd_destroy(None) == 0


def test_launch_floor_rejects_bad_arguments_without_device(lib):
    g, d = ctypes.c_double(), ctypes.c_double()
    assert lib.concpd_launch_floor(0, 10, ctypes.byref(g), ctypes.byref(d)) == 1
    assert lib.concpd_launch_floor(10, 0, ctypes.byref(g), ctypes.byref(d)) == 1
    assert lib.concpd_launch_floor(10, 10, None, ctypes.byref(d)) == 1
