"""Host-side checks of the C-ABI: the library loads, exports every symbol that
include/nlinv.h declares, and validates arguments before touching a device.
No test here launches a kernel or needs a GPU."""
import ctypes
import os

import pytest

from paper_1701_08361_amd import nlinv as nl


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nl.LIB_PATH):
        from paper_1701_08361_amd import build
        build.build(verbose=False)
    return nl.load()


def test_exports_every_header_symbol(lib):
    names = nl.header_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), f"{n} declared in nlinv.h but not exported"


@pytest.mark.parametrize("N,J,K,expect", [
    (64, 8, 13, dict(R=64, G=128, Gc=32, S=13 * 128, X=64 * 64 + 8 * 32 * 32)),
    (160, 10, 15, dict(R=160, G=320, Gc=80, S=15 * 320, X=160 * 160 + 10 * 80 * 80)),
    (224, 16, 21, dict(R=224, G=448, Gc=112, S=21 * 448, X=224 * 224 + 16 * 112 * 112)),
])
def test_sizes(lib, N, J, K, expect):
    p = nl.make_params(N, J, K)
    assert nl.sizes(p) == expect
    assert nl.workspace_size(p) > 0


def test_workspace_grows_with_batch(lib):
    a = nl.workspace_size(nl.make_params(160, 10, 15, batch=1))
    b = nl.workspace_size(nl.make_params(160, 10, 15, batch=16))
    # batch-1 plans also hold the split-gridding partial sums
    assert 4 * a < b < 17 * a


@pytest.mark.parametrize("kw,code", [
    (dict(N=100, J=8, K=13), nl.E_SIZE),           # G = 200 unsupported
    (dict(N=64, J=8, K=13, G=192), nl.E_SIZE),     # gamma 1.5, but no kernels for G = 192
    (dict(N=64, J=8, K=13, G=64), nl.E_SIZE),      # gamma < 1
    (dict(N=64, J=8, K=14), nl.E_ARG),             # even spoke count
    (dict(N=64, J=0, K=13), nl.E_ARG),
    (dict(N=64, J=65, K=13), nl.E_ARG),
    (dict(N=64, J=8, K=13, batch=0), nl.E_ARG),
    (dict(N=64, J=8, K=13, batch=65), nl.E_ARG),
    (dict(N=64, J=8, K=13, U=0), nl.E_ARG),
    (dict(N=64, J=8, K=13, cg=0), nl.E_ARG),
    (dict(N=64, J=8, K=13, flags=8), nl.E_ARG),   # unknown flag bit
    (dict(N=64, J=8, K=13, flags=1), nl.E_ARG),   # bit 1 is not a flag
    (dict(N=64, J=8, K=13, alpha0=0.0), nl.E_ARG),
    (dict(N=64, J=8, K=13, alpha_q=1.5), nl.E_ARG),
    (dict(N=64, J=8, K=13, alpha_min=-1.0), nl.E_ARG),
    (dict(N=0, J=8, K=13), nl.E_ARG),
    (dict(N=64, J=8, K=13, col_tile=2), nl.E_ARG),   # tile schedule: 0, 4 or 8
    (dict(N=64, J=8, K=13, cg_passes=5), nl.E_ARG),  # a CG iteration has 4 or 6 passes
    (dict(N=64, J=8, K=13, fft_split=2), nl.E_ARG),  # factorisations 0 and 1
])
def test_invalid_params_rejected(lib, kw, code):
    p = nl.make_params(**kw)
    with pytest.raises(nl.NlinvError) as ei:
        nl.workspace_size(p)
    assert ei.value.code == code
    assert len(lib.nlinv_last_error(None)) > 0


def test_plan_create_checks_workspace_before_any_device_call(lib):
    p = nl.make_params(64, 8, 13)
    need = nl.workspace_size(p)
    h = ctypes.c_void_p()
    rc = lib.nlinv_plan_create(ctypes.byref(p), None, None, need, ctypes.byref(h))
    assert rc == nl.E_WORKSPACE and not h.value
    rc = lib.nlinv_plan_create(ctypes.byref(p), None, ctypes.c_void_p(1 << 20), need - 1, ctypes.byref(h))
    assert rc == nl.E_WORKSPACE
    rc = lib.nlinv_plan_create(ctypes.byref(p), None, ctypes.c_void_p((1 << 20) + 8), need, ctypes.byref(h))
    assert rc == nl.E_WORKSPACE and b"aligned" in lib.nlinv_last_error(None)
    assert lib.nlinv_plan_create(ctypes.byref(p), None, None, 0, None) == nl.E_ARG


def test_null_plan_rejected(lib):
    assert lib.nlinv_sync(None) == nl.E_ARG
    assert lib.nlinv_reconstruct(None, None, None, None, None, 1, None, None) == nl.E_ARG
    assert lib.nlinv_grid(None, None, None, None, None) == nl.E_ARG
    assert lib.nlinv_plan_destroy(None) == nl.E_ARG
    assert lib.nlinv_reconstruct_frames(None, 1, None, None, None, None, None, None) == nl.E_ARG
    assert lib.nlinv_set_batch(None, 1) == nl.E_ARG
    assert lib.nlinv_psf(None, None, 0) == nl.E_ARG
    assert lib.nlinv_psf_spokes(None, None, 1, 0) == nl.E_ARG
    assert lib.nlinv_psf_samples(None, None, 1, 0) == nl.E_ARG
    assert lib.nlinv_get_batch(None) == 0
    assert b"NULL" in lib.nlinv_last_error(None)
    # the entry points of the differentiable form and of the multi-plan operator
    assert lib.nlinv_newton_step(None, None, None, None, 0.5, 4, None) == nl.E_ARG
    assert lib.nlinv_set_coil_weights(None, None) == nl.E_ARG
    assert lib.nlinv_apply_normal2(None, None, None, None, 0.0, None, None) == nl.E_ARG
    assert lib.nlinv_apply_E(None, None, None, None) == nl.E_ARG
    assert lib.nlinv_apply_EH(None, None, None, None) == nl.E_ARG
    assert lib.nlinv_nudft(None, None, None, None) == nl.E_ARG
    assert lib.nlinv_apply_normal_multi(0, None, None, None, None, None, None) == nl.E_ARG
    assert lib.nlinv_apply_normal_multi(4, None, None, None, None, None, None) == nl.E_ARG
    assert lib.nlinv_apply_normal_multi(1, None, None, None, None, None, None) == nl.E_ARG
    assert b"NULL" in lib.nlinv_last_error(None)
    one = (ctypes.c_void_p * 1)(None)
    arr = (ctypes.c_void_p * 1)(None)
    alpha = (ctypes.c_double * 1)(0.0)
    assert lib.nlinv_apply_normal_multi(1, one, arr, arr, alpha, arr, arr) == nl.E_ARG
    # the one-launch multi-plan reconstruction
    inits = (ctypes.c_int32 * 1)(1)
    assert lib.nlinv_reconstruct_multi(0, None, None, None, None, None, None, None) == nl.E_ARG
    assert lib.nlinv_reconstruct_multi(9, None, None, None, None, None, None, None) == nl.E_ARG
    assert lib.nlinv_reconstruct_multi(1, None, None, None, None, None, None, None) == nl.E_ARG
    assert lib.nlinv_reconstruct_multi(1, one, arr, arr, arr, arr, inits, arr) == nl.E_ARG


def test_static_plan_rejects_oversized_parameters(lib):
    """nlinv_plan_create_static checks the workspace size against the static
    array before any device call."""
    p = nl.make_params(256, 64, 21, U=8, batch=4)
    assert nl.workspace_size(p) > nl.STATIC_WORKSPACE_BYTES
    h = ctypes.c_void_p()
    assert lib.nlinv_plan_create_static(ctypes.byref(p), None, ctypes.byref(h)) == nl.E_WORKSPACE
    assert not h.value and b"static workspace" in lib.nlinv_last_error(None)
    assert lib.nlinv_plan_create_static(ctypes.byref(p), None, None) == nl.E_ARG
