"""C-ABI contract on the CPU: the library loads, exports every declared entry
point, and its host-side argument checks and planning work without a GPU
(no compute call is made here)."""
import ctypes
import math
import os
import re

import pytest

import paper_2306_12616_amd as chebdm
from paper_2306_12616_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "chebdm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chebdm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(chebdm.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return chebdm.load_library()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared_symbols()
    assert declared, "header parse found no entry points"
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(_binding.EXPORTED)


def test_abi_version_and_defaults(lib):
    assert lib.chebdm_abi_version() == 4
    o = chebdm.make_opts()
    assert (o.prec, o.giant_form, o.k_override, o.n_quad, o.max_iter, o.baby_steps, o.search, o.damping, o.tol) == \
        (0, 0, 0, 0, 200, 0, 0, 0, 1e-10)
    assert chebdm.make_opts(damping="jackson").damping == 1
    assert ctypes.sizeof(chebdm.Opts) == 56   # eight int32, a double, two int32, a double
    assert chebdm.make_opts(search="newton").search == 1
    assert (o.bounds, o.lanczos_steps, o.bounds_margin) == (0, 0, 0.0)
    lz = chebdm.make_opts(bounds="lanczos", lanczos_steps=24, bounds_margin=0.05)
    assert (lz.bounds, lz.lanczos_steps, lz.bounds_margin) == (1, 24, 0.05)


def test_bounds_options_are_checked_on_the_host(lib):
    # chebdm_workspace_size validates the options without touching a device
    size = ctypes.c_size_t()
    for kw in ({"bounds": 2}, {"bounds": -1}, {"bounds": "lanczos", "lanczos_steps": 129},
               {"bounds": "lanczos", "lanczos_steps": -1}, {"bounds": "lanczos", "bounds_margin": -0.1},
               {"bounds": "lanczos", "bounds_margin": math.inf}):
        o = chebdm.make_opts(**kw)
        assert lib.chebdm_workspace_size(None, 100, 64, ctypes.byref(o), ctypes.byref(size)) == _binding.ERR_ARG, kw
    o = chebdm.make_opts(bounds="lanczos", lanczos_steps=128, bounds_margin=0.5)
    assert lib.chebdm_workspace_size(None, 100, 64, ctypes.byref(o), ctypes.byref(size)) == 0


def _dbl():
    return ctypes.c_double()


def test_null_handle_is_rejected(lib):
    lo, hi = _dbl(), _dbl()
    assert lib.chebdm_bounds(None, None, 4, 4, ctypes.byref(lo), ctypes.byref(hi)) == _binding.ERR_ARG
    c = (ctypes.c_double * 8)()
    assert lib.chebdm_coeffs(None, 1.0, 0.0, -1.0, 1.0, 7, 0, c) == _binding.ERR_ARG
    assert lib.chebdm_density(None, None, 4, 4, 1.0, 0.0, 4, None, math.nan, math.nan, None, 4, None) == _binding.ERR_ARG
    mu = _dbl()
    assert lib.chebdm_mu_search(None, None, 4, 4, 1.0, 2.0, 4, None, math.nan, math.nan, ctypes.byref(mu), None, 4,
                                None) == _binding.ERR_ARG
    assert lib.chebdm_moments(None, None, 4, 4, 4, None, math.nan, math.nan, c) == _binding.ERR_ARG
    assert lib.chebdm_bounds_lanczos(None, None, 4, 4, 8, 0.01, 0, ctypes.byref(lo), ctypes.byref(hi), None, None,
                                     None) == _binding.ERR_ARG
    assert lib.chebdm_commutator_norm(None, None, 4, None, 4, 4, ctypes.byref(lo)) == _binding.ERR_ARG
    assert b"NULL" in lib.chebdm_last_error() or b"handle" in lib.chebdm_last_error()
    assert lib.chebdm_destroy(None) == 0
    assert lib.chebdm_set_stream(None, None) == _binding.ERR_ARG


@pytest.mark.parametrize("order,k,m", [(128, 12, 11), (512, 23, 23), (256, 17, 16), (2048, 46, 45), (0, 1, 1),
                                       (24, 5, 5), (1, 2, 1)])
def test_block_split_matches_plan(lib, order, k, m):
    # the size query of chebdm_block_coeffs is host-only planning
    kk, mm = ctypes.c_int32(), ctypes.c_int32()
    dummy = ctypes.c_void_p(1)
    rc = lib.chebdm_block_coeffs(dummy, None, order, 0, 0, ctypes.byref(kk), ctypes.byref(mm), None)
    assert rc == 0 and (kk.value, mm.value) == (k, m)


def test_block_split_override_and_limits(lib):
    kk, mm = ctypes.c_int32(), ctypes.c_int32()
    dummy = ctypes.c_void_p(1)
    assert lib.chebdm_block_coeffs(dummy, None, 100, 0, 7, ctypes.byref(kk), ctypes.byref(mm), None) == 0
    assert (kk.value, mm.value) == (7, 15)
    # more than 48 blocks is refused
    assert lib.chebdm_block_coeffs(dummy, None, 2048, 0, 4, ctypes.byref(kk), ctypes.byref(mm), None) == _binding.ERR_ARG
    assert lib.chebdm_block_coeffs(dummy, None, 48 * 48, 0, 0, ctypes.byref(kk), ctypes.byref(mm), None) == _binding.ERR_ARG
    assert lib.chebdm_block_coeffs(dummy, None, -1, 0, 0, ctypes.byref(kk), ctypes.byref(mm), None) == _binding.ERR_ARG
    assert lib.chebdm_block_coeffs(dummy, None, 10, 5, 0, ctypes.byref(kk), ctypes.byref(mm), None) == _binding.ERR_ARG


def test_workspace_size_needs_no_device(lib):
    # (k + m + 1) ld^2 elements plus the small buffers; k = m = 23 at order 512, ld = 4096 at
    # n = 4000 (the extra matrix is T_h(T_k) of the two-chain giant steps, the library's choice at
    # this size; four chains keep T_q(T_k) too, one chain and the power form neither)
    small = chebdm.chebdm_workspace_size(1, 0)
    f64 = chebdm.chebdm_workspace_size(4000, 512)
    f32 = chebdm.chebdm_workspace_size(4000, 512, chebdm.make_opts("fp32"))
    power = chebdm.chebdm_workspace_size(4000, 512, chebdm.make_opts("fp64", "power"))
    four = chebdm.chebdm_workspace_size(4000, 512, chebdm.make_opts("fp64", "four_chains"))
    one = chebdm.chebdm_workspace_size(4000, 512, chebdm.make_opts("fp64", "one_chain"))
    assert f64 - small >= 47 * 4096 * 4096 * 8 - 2 * 128 * 128 * 8
    assert f64 - f32 == 47 * 4096 * 4096 * 4
    assert four - f64 == 4096 * 4096 * 8 and f64 - one == 4096 * 4096 * 8
    assert f64 - power == 4096 * 4096 * 8
    # at n = 2000 (528 64-tiles per product) the library takes four chains
    f64_2k = chebdm.chebdm_workspace_size(2000, 512)
    one_2k = chebdm.chebdm_workspace_size(2000, 512, chebdm.make_opts("fp64", "one_chain"))
    assert f64_2k - one_2k == 2 * 2048 * 2048 * 8
    with pytest.raises(chebdm.ChebdmError):
        chebdm.chebdm_workspace_size(0, 10)
