"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1610_05329_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgpe.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dgpe_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdgpe.so is not built (python -m paper_1610_05329_amd.build)")
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def _n(*v):
    return (ctypes.c_int32 * 3)(*v)


def test_workspace_bytes_accepts_fft_friendly_sizes(lib):
    for n in [(32, 32, 32), (96, 96, 96), (256, 256, 256), (512, 512, 256), (12, 18, 24), (4, 4, 4)]:
        for mode in (0, 1, 2, 3):
            assert lib.dgpe_workspace_bytes(_n(*n), mode) > 0, (n, mode)


@pytest.mark.parametrize("bad", [(10, 32, 32), (32, 5, 32), (32, 32, 7), (4096, 32, 32), (2, 8, 8), (40, 40, 40),
                                 (2048, 2048, 512)])  # the last: more than 2^30 points
def test_workspace_bytes_rejects_other_sizes(lib, bad):
    assert lib.dgpe_workspace_bytes(_n(*bad), 0) == 0


def test_workspace_holds_half_spectrum_not_full(lib):
    # R2C along z: the spectrum needs Nx Ny (Nz/2+1) complex values (paper,
    # "Summary of revisions": half the values of the Hermitian spectrum)
    n = (64, 64, 64)
    ws = lib.dgpe_workspace_bytes(_n(*n), 0)
    full_spectrum = 64 ** 3 * 16
    state = 64 ** 3 * 16
    half = 64 * 64 * 33 * 16
    assert ws >= half
    assert ws < full_spectrum + state // 2 + half  # spectrum + one real buffer + tables


def _create(lib, n=(32, 32, 32), d=(0.25,) * 3, dt=0.005, trap=(1.0, 1.0, 1.0), g=1.0, gd=1.0,
            mode=0, ws=None, nbytes=0):
    h = ctypes.c_void_p()
    st = lib.dgpe_plan_create(ctypes.byref(h), _n(*n), (ctypes.c_double * 3)(*d), dt,
                              (ctypes.c_double * 3)(*trap), g, gd, 0.0, mode, ws, nbytes, None)
    return st, h


def test_plan_create_validates_before_device_work(lib):
    st, h = _create(lib, n=(30, 32, 32))
    assert st == 2 and not h.value
    assert b"2^a 3^b" in lib.dgpe_last_error()
    assert _create(lib, dt=0.0)[0] == 1
    assert _create(lib, dt=float("nan"))[0] == 1
    assert _create(lib, d=(0.25, -1.0, 0.25))[0] == 1
    assert _create(lib, g=float("inf"))[0] == 1
    assert _create(lib, mode=16)[0] == 1  # an unknown mode bit
    assert _create(lib, ws=None)[0] == 3
    assert _create(lib, ws=ctypes.c_void_p(0x1000 + 8), nbytes=1 << 40)[0] == 3
    assert _create(lib, ws=ctypes.c_void_p(0x1000), nbytes=16)[0] == 3
    assert b"too small" in lib.dgpe_last_error()


def test_null_plan_calls_fail_cleanly(lib):
    assert lib.dgpe_step(None, None, 1, None) == 1
    assert lib.dgpe_plan_set(None, 0, 1.0) == 1
    assert lib.dgpe_adjoint_workspace_bytes(None, 10, 2) == 0
    lib.dgpe_plan_destroy(None)
    assert lib.dgpe_status_string(5) == b"DGPE_ENONFINITE"
    assert lib.dgpe_status_string(0) == b"DGPE_OK"


def test_schedule_query_rejects_null_plan(lib):
    assert lib.dgpe_plan_fused_y(None) == -1


def test_noalloc_plan_rejects_grids_beyond_its_scratch_before_device_work(lib):
    """The allocation-free plan checks its arguments and the 64 MiB limit of its
    static scratch before any HIP call (so this runs without a GPU)."""
    def create(n, mode=0, dt=0.005):
        h = ctypes.c_void_p()
        st = lib.dgpe_plan_create_noalloc(ctypes.byref(h), _n(*n), (ctypes.c_double * 3)(0.2, 0.2, 0.2),
                                          dt, (ctypes.c_double * 3)(1.0, 1.0, 1.0), 1.0, 1.0, 0.0,
                                          mode, None)
        return st, h
    assert _lib.NOALLOC_MAX_BYTES == 64 << 20
    # 192^3 FP64 needs about 116 MiB; 256^3 FP32 about 137 MiB
    for n, mode in [((192, 192, 192), 0), ((256, 256, 256), 2)]:
        assert lib.dgpe_workspace_bytes(_n(*n), mode) > _lib.NOALLOC_MAX_BYTES
        st, h = create(n, mode)
        assert st == 3 and not h.value
        assert b"at most" in lib.dgpe_last_error()
    assert create((30, 32, 32))[0] == 2
    assert create((32, 32, 32), dt=-1.0)[0] == 1
    h = ctypes.c_void_p()
    assert lib.dgpe_plan_create_noalloc(None, _n(32, 32, 32), (ctypes.c_double * 3)(0.2, 0.2, 0.2),
                                        0.005, (ctypes.c_double * 3)(1.0, 1.0, 1.0), 1.0, 1.0,
                                        0.0, 0, None) == 1
    # the largest grids it serves fit the limit
    assert lib.dgpe_workspace_bytes(_n(128, 128, 128), 0) <= _lib.NOALLOC_MAX_BYTES
    assert lib.dgpe_workspace_bytes(_n(192, 192, 192), 2) <= _lib.NOALLOC_MAX_BYTES


def test_quasi2d_mode_validation_before_device_work(lib):
    """Quasi-2D plans: the grid is (N1, 1, N2), one orientation bit, a positive
    tight trap frequency; everything else is refused before any HIP call."""
    PERP, INPLANE = _lib.Q2D["perp"], _lib.Q2D["inplane"]
    assert lib.dgpe_workspace_bytes(_n(64, 1, 48), PERP) > 0
    assert lib.dgpe_workspace_bytes(_n(64, 1, 48), INPLANE | 3) > 0
    assert lib.dgpe_workspace_bytes(_n(64, 1, 48), 0) == 0          # 3D needs Ny >= 4
    assert lib.dgpe_workspace_bytes(_n(64, 4, 48), PERP) == 0       # quasi-2D needs Ny = 1
    assert lib.dgpe_workspace_bytes(_n(64, 1, 48), PERP | INPLANE) == 0
    assert lib.dgpe_workspace_bytes(_n(64, 1, 50), PERP) == 0       # 50 = 2 * 5^2

    def create(n, mode, trap=(1.0, 4.0, 1.0)):
        h = ctypes.c_void_p()
        return lib.dgpe_plan_create(ctypes.byref(h), _n(*n), (ctypes.c_double * 3)(0.3, 1.0, 0.3), 0.01,
                                    (ctypes.c_double * 3)(*trap), 1.0, 1.0, 0.0, mode, None, 0, None)
    assert create((32, 2, 32), PERP) == 2
    assert create((32, 1, 32), PERP | INPLANE) == 1
    assert create((32, 1, 32), PERP, trap=(1.0, 0.0, 1.0)) == 1
    assert create((32, 1, 32), INPLANE, trap=(1.0, -2.0, 1.0)) == 1
    assert create((32, 1, 32), PERP) == 3  # valid arguments: then the missing workspace
