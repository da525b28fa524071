"""CPU-side checks of the C ABI: the built library loads and exports every
function include/sps.h declares, and the binding wraps each under the same
name.  No compute calls are made (no GPU here)."""
import ctypes
import os

import pytest

from paper_2511_02328_amd.build import LIB_PATH


def _header_functions():
    from paper_2511_02328_amd import sps
    return sps.header_functions()


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB_PATH):
        pytest.fail("HIP library not built: run __graft_entry__.build()")
    import torch  # noqa: F401  (binds the HIP runtime torch ships first)
    return ctypes.CDLL(LIB_PATH)


def test_header_declares_the_boundary():
    names = _header_functions()
    for required in ("sps_plan_create", "sps_plan_destroy", "sps_plan_delays", "sps_dedisperse",
                     "sps_boxcar_snr", "sps_detect", "sps_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _header_functions():
        assert hasattr(lib, name), f"{name} declared in sps.h but not exported"


def test_binding_uses_the_same_names(lib):
    from paper_2511_02328_amd import sps
    for name in _header_functions():
        assert callable(getattr(sps, name, None)), f"binding lacks {name}"


def test_last_error_is_empty_string_initially(lib):
    lib.sps_last_error.restype = ctypes.c_char_p
    assert lib.sps_last_error() == b""


def test_null_arguments_fail_before_touching_a_device(lib):
    # validation happens before any HIP call, so these run without a GPU
    lib.sps_plan_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    out = ctypes.c_void_p(1)
    assert lib.sps_plan_create(None, ctypes.byref(out)) == 1
    assert out.value is None
    lib.sps_dedisperse.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_uint32, ctypes.c_void_p]
    assert lib.sps_dedisperse(None, None, 16, 16, None, 1, 0, None) == 1
    lib.sps_plan_destroy.argtypes = [ctypes.c_void_p]
    assert lib.sps_plan_destroy(None) == 0
    lib.sps_probe_peaks.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32]
    assert lib.sps_probe_peaks(0, None, 4) == 1
    rates = (ctypes.c_double * 4)()
    assert lib.sps_probe_peaks(0, rates, 4) == 1


def test_no_cpu_fallback_in_the_product_package():
    # the product package never imports the oracle
    pkg = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2511_02328_amd")
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(root, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "sps_oracle" not in text, f


def test_oracle_and_inputs_never_import_the_product_package():
    # the oracle shares no code with the HIP path, and the shared seeded-input
    # package imports neither side
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for sub in ("oracle", "sps_inputs"):
        for dirpath, _, files in os.walk(os.path.join(root, sub)):
            for f in files:
                if f.endswith((".py", ".c", ".h")):
                    text = open(os.path.join(dirpath, f)).read()
                    assert "paper_2511_02328_amd" not in text.replace(
                        "(``paper_2511_02328_amd``)", ""), os.path.join(sub, f)
                    if sub == "sps_inputs":
                        assert "import oracle" not in text and "from oracle" not in text, f
