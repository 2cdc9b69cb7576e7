"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function that include/scsc.h declares, and its host-only helpers agree with the
binding's layout logic."""

import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scsc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1909_00145_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libscsc.so is not built: run python -m paper_1909_00145_amd.build")
    return _lib.lib()


def test_exports_every_declared_symbol(lib):
    from paper_1909_00145_amd import _lib

    names = declared_functions()
    assert "csc_code_step" in names and "csc_dict_step" in names and "csc_objective" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_version(lib):
    assert lib.csc_version() == 100


def test_surrogate_layout_is_a_permutation(lib):
    from paper_1909_00145_amd.ops import lag_index_map

    for K, m in [(1, 3), (2, 5), (3, 3)]:
        assert lib.csc_surrogate_size(K, m) == (K * m * m) ** 2
        idx = lag_index_map(K, m)
        np.testing.assert_array_equal(np.sort(idx.ravel()), np.arange((K * m * m) ** 2))
        c = m // 2
        M = m * m
        for i in range(0, K * M, 3):
            for j in range(0, K * M, 2):
                k, s = divmod(i, M)
                k2, s2 = divmod(j, M)
                assert lib.csc_surrogate_index(K, m, k, s // m - c, s % m - c, k2, s2 // m - c, s2 % m - c) == idx[i, j]


def test_surrogate_index_rejects_bad_arguments(lib):
    assert lib.csc_surrogate_index(2, 5, 2, 0, 0, 0, 0, 0) == -1
    assert lib.csc_surrogate_index(2, 5, 0, 3, 0, 0, 0, 0) == -1
    assert lib.csc_surrogate_index(2, 4, 0, 0, 0, 0, 0, 0) == -1
    assert lib.csc_surrogate_size(0, 3) == -1


def test_null_handle_is_rejected(lib):
    from paper_1909_00145_amd import _lib

    assert lib.csc_destroy(None) == _lib.CSC_EINVAL
    assert lib.csc_code_step(None, None, None, None, None, 1, 3, None, 1.0, 0.5, 0, 0, 1, 0.0, 0, None) == _lib.CSC_EINVAL
    assert lib.csc_last_error(None) == b"null handle"
