"""The C-ABI surface on the CPU: the library loads, exports every declared entry point, and the
binding fails loudly (no CPU fallback) when no GPU is present."""

import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "omm.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(omm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def libomm():
    from paper_1312_1549_amd import _lib

    if not _lib.LIB_PATH.exists():
        from paper_1312_1549_amd.build import build

        build()
    return _lib.lib()


def test_header_declares_the_paper_calls():
    names = declared_functions()
    for required in ("omm_create", "omm_set_HS", "omm_minimize", "omm_energy", "omm_density",
                     "omm_edm", "omm_backward_device", "omm_batch_minimize"):
        assert required in names


def test_every_declared_symbol_is_exported(libomm):
    from paper_1312_1549_amd._lib import PROTOTYPES

    names = declared_functions()
    assert set(names) == set(PROTOTYPES)
    for n in names:
        assert hasattr(libomm, n), n


def test_argument_errors_need_no_gpu(libomm):
    import ctypes as ct

    h = ct.c_void_p()
    assert libomm.omm_create(10, 11, ct.byref(h)) == -1  # M > N
    assert libomm.omm_create(0, 0, ct.byref(h)) == -1
    assert libomm.omm_create(10, 2, None) == -1
    assert libomm.omm_destroy(None) == -1
    assert libomm.omm_last_error(None) == b"null context"
    N = (ct.c_int64 * 2)(64, 64)
    M = (ct.c_int64 * 2)(8, 65)
    assert libomm.omm_batch_create_complex(2, N, M, ct.byref(h)) == -1  # M > N
    assert libomm.omm_batch_create_complex(0, N, M, ct.byref(h)) == -1
    big = (ct.c_int64 * 1)(1 << 16)
    assert libomm.omm_batch_create_complex(1, big, M, ct.byref(h)) == -1
    assert libomm.omm_create_complex(10, 11, ct.byref(h)) == -1


def test_no_silent_cpu_fallback(libomm):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1312_1549_amd import OMM, OMMError

    with pytest.raises(OMMError):
        OMM(128, 24)
