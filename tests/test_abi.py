"""The C-ABI library loads on a machine without a GPU and exports every symbol that
include/smc.h declares; the Python binding covers the same names (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smc.h")
LIB = os.path.join(ROOT, "paper_2601_21983_amd", "libsmc.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:SMC_API\s+)?(?:const\s+)?[a-z_0-9]+\s*\*?\s*(smc_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import importlib.util
        spec = importlib.util.spec_from_file_location("smc_build", os.path.join(ROOT, "paper_2601_21983_amd", "build.py"))
        m = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(m)
        m.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["smc_init", "smc_step", "smc_resample", "smc_posterior_predict", "smc_destroy",
                     "smc_get_state", "smc_set_state", "smc_set_noise", "smc_set_proposal_net",
                     "smc_nn_forward", "smc_nn_backward", "smc_status_string"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_gpu(lib):
    lib.smc_status_string.restype = ctypes.c_char_p
    assert lib.smc_status_string(0) == b"ok"
    assert b"argument" in lib.smc_status_string(1)


def test_null_arguments_are_rejected_without_gpu(lib):
    # argument validation happens before any device call
    lib.smc_init.restype = ctypes.c_int32
    out = ctypes.c_void_p()
    assert lib.smc_init(None, None, None, ctypes.c_int64(0), None, ctypes.c_int64(0), ctypes.c_double(1.0), None,
                        ctypes.byref(out)) == 1
    assert out.value is None


def test_binding_names_match_header():
    from paper_2601_21983_amd import _lib
    assert sorted(_lib.EXPORTED) == _declared()
    for n in _declared():
        assert callable(getattr(_lib, n))


def test_binding_constants_match_header_enums():
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    values = {}
    for body in re.findall(r"enum\s*(?:[a-z_]+\s*)?\{([^}]*)\}", src):
        for name, val in re.findall(r"(SMC_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            values[name] = int(val)
    from paper_2601_21983_amd import _lib
    checked = [n for n in values if hasattr(_lib, n)]
    assert {"SMC_MODEL_MLP", "SMC_MODEL_CNN", "SMC_MODEL_LENET"} <= set(checked)
    for n in checked:
        assert getattr(_lib, n) == values[n], n


def test_parameter_counts_match_the_oracle():
    from oracle import cnn, lenet, mlp
    from paper_2601_21983_amd.sampler import n_params
    assert n_params(list(lenet.LENET5_MNIST), "lenet") == lenet.LeNetShape(*lenet.LENET5_MNIST).D == 61706
    for shape in [(12, 12, 1, 5, 3, 4, 8, 8, 3), (12, 12, 2, 3, 3, 5, 8, 4, 3), (8, 12, 2, 3, 5, 6, 8, 4, 4)]:
        assert n_params(list(shape), "lenet") == lenet.LeNetShape(*shape).D
    assert n_params([32, 32, 3, 16, 32, 10], "cnn") == cnn.CNNShape(32, 32, 3, 16, 32, 10).D
    assert n_params([784, 100, 10]) == mlp.n_params([784, 100, 10])
