"""The C-ABI library loads and exports every symbol its header declares, and its
host-side validation returns the documented status codes.  No GPU is touched:
only calls that fail before any HIP call (or never make one) are used."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(pic_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1011_6330_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        from paper_1011_6330_amd import build
        build.build()
    return _binding.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    from paper_1011_6330_amd import _binding
    assert set(names) == set(_binding.SIGNATURES), set(names) ^ set(_binding.SIGNATURES)


def test_abi_version(lib):
    from paper_1011_6330_amd import _binding
    m = re.search(r"#define PCPIC_ABI_VERSION (\d+)", open(os.path.join(ROOT, "include", "pcpic.h")).read())
    assert lib.pic_abi_version() == int(m.group(1)) == _binding.ABI_VERSION == 4


def _params(**kw):
    from paper_1011_6330_amd import _binding
    p, k, _ = _binding.make_params(kw)
    return p, k


def test_workspace_bytes_and_validation(lib):
    p, _k = _params()
    n = lib.pic_workspace_bytes(ctypes.byref(p))
    # two FP64 particle buffers of 65536 slots dominate
    assert n >= 4 * 8 * (1 << 16)
    big, _k2 = _params(capacity=1 << 20)
    assert lib.pic_workspace_bytes(ctypes.byref(big)) > n
    bad, _k3 = _params(dt_over_dz=1.0)
    assert lib.pic_workspace_bytes(ctypes.byref(bad)) == 0
    assert b"dt_over_dz" in lib.pic_last_error()


@pytest.mark.parametrize("kw,code", [
    (dict(dt_over_dz=1.2), -5),          # PIC_ECFL
    (dict(n_cells=1), -1),               # PIC_EINVAL
    (dict(ppc=0.0), -1),
    (dict(rho_kind=2), -1),              # knots missing
    (dict(fp_bits=50), -1),
])
def test_init_rejects_bad_params(lib, kw, code):
    p, _k = _params(**kw)
    h = ctypes.c_void_p()
    rc = lib.pic_init(ctypes.byref(p), None, 0, None, ctypes.byref(h))
    assert rc == code and not h.value


def test_init_rejects_bad_abi_and_workspace(lib):
    p, _k = _params()
    p.abi_version = 99
    h = ctypes.c_void_p()
    assert lib.pic_init(ctypes.byref(p), None, 0, None, ctypes.byref(h)) == -8     # PIC_EABI
    p.abi_version = lib.pic_abi_version()
    assert lib.pic_init(ctypes.byref(p), None, 0, None, ctypes.byref(h)) == -2     # PIC_EWORKSPACE
    assert lib.pic_init(ctypes.byref(p), ctypes.c_void_p(8), 1 << 40, None, ctypes.byref(h)) == -2  # misaligned
    assert b"aligned" in lib.pic_last_error()


def test_null_handle_calls(lib):
    assert lib.pic_step(None, 1) == -1
    assert lib.pic_sync(None) == -1
    assert lib.pic_destroy(None) == -1


def test_stream_copy_validates_before_launching(lib):
    """The benchmark's copy helper rejects bad requests on the host (these
    addresses are never dereferenced: every case fails or is empty before any
    HIP call)."""
    P = ctypes.c_void_p
    assert lib.pic_stream_copy(None, P(4096), 16, None) == -1
    assert lib.pic_stream_copy(P(4104), P(8192), 16, None) == -1       # source not 16-byte aligned
    assert lib.pic_stream_copy(P(4096), P(8192), 24, None) == -1       # size not a multiple of 16
    assert lib.pic_stream_copy(P(4096), P(4160), 128, None) == -1      # ranges overlap
    assert lib.pic_stream_copy(P(4096), P(8192), 1 << 40, None) == -1  # too large
    assert lib.pic_stream_copy(P(4096), P(8192), 0, None) == 0         # nothing to do
