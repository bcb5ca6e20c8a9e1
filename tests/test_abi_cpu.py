"""CPU checks of the C ABI boundary: the library loads and exports every
symbol declared in include/ihsbin.h, and its host-only calls behave."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ihsbin.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ihsbin_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2210_12212_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    from paper_2210_12212_amd import _lib
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(_lib.EXPORTED)


def test_status_strings_and_version(lib):
    assert lib.ihsbin_status_str(0) == b"ok"
    assert b"range" in lib.ihsbin_status_str(-6)
    assert lib.ihsbin_version().startswith(b"ihsbin")


def test_default_options(lib):
    from paper_2210_12212_amd import _lib
    o = _lib.Opts()
    lib.ihsbin_opts_default(C.byref(o))
    assert o.tol == 1e-8 and o.k_max == 96 and o.centred == 1 and o.adaptive_m == 1
    assert o.lanczos_steps == 12 and not o.taus
    assert o.basis_prec == 0 and o.f32_switch == 1e-2 and o.graph_steps == 0


def test_null_arguments_are_rejected(lib):
    assert lib.ihsbin_create(None, 0, None) == -1
    assert lib.ihsbin_path_free(None) == 0
    assert lib.ihsbin_destroy(None) == 0
    assert lib.ihsbin_path_build(None, None, None, 1, 1, 1.0, 2.0, None, None, None) == -1
    assert lib.ihsbin_last_error(None) == b""


def test_struct_sizes_match_header_layout():
    from paper_2210_12212_amd import _lib
    # int32 x2, int64 x4, pointers x3
    assert C.sizeof(_lib.Matrix) == 8 + 32 + 24
    assert C.sizeof(_lib.PathInfo) == 4 + 4 + 8 + 8 + 8 + 8 + 4 + 4  # ..., centred, dual
    assert C.sizeof(_lib.Alg4Opts) == 4 * 8 + 4 + 4
    assert C.sizeof(_lib.Alg4Result) == 8 + 4 + 4 + 3 * 8


def test_alg4_default_options(lib):
    from paper_2210_12212_amd import _lib
    a = _lib.Alg4Opts()
    lib.ihsbin_alg4_opts_default(C.byref(a))
    assert (a.gamma1, a.gamma2, a.gamma3, a.eps) == (0.5, 1e-4, 0.5, 1e-8)
    assert a.max_iter == 50 and a.max_armijo == 60
    o = _lib.Opts()
    lib.ihsbin_opts_default(C.byref(o))
    assert not o.alg4


def test_serving_struct_sizes():
    from paper_2210_12212_amd import _lib
    assert C.sizeof(_lib.ServerOpts) == 4 + 4 + 8 + 8
    assert C.sizeof(_lib.ServerStats) == 3 * 8 + 4 * 4 + 3 * 8
    assert C.sizeof(_lib.RequestInfo) == 4 + 4 + 8 + 3 * 8 + C.sizeof(_lib.Report) + 160


def test_footprint_estimate_host_only(lib):
    # no device is touched: only shapes and options enter the estimate
    from paper_2210_12212_amd import build_footprint
    f1 = build_footprint((100000, 1024), 1, 1e-4, 10.0, sketch="srht")
    f2 = build_footprint((200000, 1024), 1, 1e-4, 10.0, sketch="srht")
    f3 = build_footprint((100000, 2048), 1, 1e-4, 10.0, sketch="srht")
    f4 = build_footprint((100000, 1024), 8, 1e-4, 10.0, sketch="srht")
    assert 0 < f1 < f2 and f1 < f3 and f1 < f4
    # the factors alone: 2 L d^2 doubles, L = 23
    assert f3 >= 2 * 23 * 2048 * 2048 * 8
    fd = build_footprint((500, 20000), 1, 1e-2, 10.0, sketch="gaussian")  # dual
    assert fd >= 500 * 20000 * 4
    from paper_2210_12212_amd import IhsbinError
    with pytest.raises(IhsbinError):
        build_footprint((100, 10), 1, 0.0, 1.0)


def test_report_layout():
    from paper_2210_12212_amd import _lib
    # int64, int32 x6, double x5, int64, double x4, int64, double, int64,
    # double x3, double
    assert C.sizeof(_lib.Report) == 8 + 6 * 4 + 5 * 8 + 8 + 4 * 8 + 8 + 8 + 8 + 3 * 8 + 8


@pytest.mark.parametrize("n,m,s", [(1000, 37, 1), (4099, 64, 4), (1, 5, 1), (70000, 4096, 1),
                                   (3000, 96, 3)])
def test_host_countsketch_draws_match_oracle(lib, n, m, s):
    # the library's host draws against the oracle's independent SplitMix64
    from oracle import rng
    from paper_2210_12212_amd import sketch_indices_host
    kind = "sjlt" if s > 1 else "countsketch"
    idx, sign = sketch_indices_host(2024 + n, kind, n, m, s)
    h, sg = rng.countsketch_draws(2024 + n, n, m, s)
    assert np.array_equal(idx.reshape(h.shape), h)
    assert np.array_equal(sign.reshape(sg.shape), sg)


@pytest.mark.parametrize("n,m", [(1000, 100), (4096, 333), (3, 7), (131072, 1024)])
def test_host_srht_draws_match_oracle(lib, n, m):
    from oracle import rng
    from paper_2210_12212_amd import sketch_indices_host
    rows, sign = sketch_indices_host(99 + m, "srht", n, m)
    sg, rr, _ = rng.srht_draws(99 + m, n, m)
    assert np.array_equal(sign, sg)
    assert np.array_equal(rows, rr)


def test_host_draws_reject_bad_arguments(lib):
    from paper_2210_12212_amd import IhsbinError, sketch_indices_host
    with pytest.raises(IhsbinError):
        sketch_indices_host(1, "gaussian", 10, 4)
    with pytest.raises(IhsbinError):
        sketch_indices_host(1, "sjlt", 10, 7, 2)     # s does not divide m
    assert lib.ihsbin_sketch_indices_host(1, 2, 10, 4, 1, None, None) == -1
