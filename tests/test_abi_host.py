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


def test_surrogate_layout_covers_the_upper_blocks_once(lib):
    """Blocks (k, k2 >= k) are stored; every stored position holds one entry of the
    upper blocks, and for k != k2 entry (k, s; k2, s2) shares its position with
    (k2, s2; k, s) (a diagonal block keeps all of its entries)."""
    from paper_1909_00145_amd.ops import lag_index_map

    for K, m in [(1, 3), (2, 5), (3, 3), (4, 5)]:
        M = m * m
        size = K * (K + 1) // 2 * M * M
        assert lib.csc_surrogate_size(K, m) == size
        idx = lag_index_map(K, m)
        off = np.kron(1 - np.eye(K, dtype=np.int64), np.ones((M, M), dtype=np.int64)).astype(bool)
        np.testing.assert_array_equal(idx[off], idx.T[off])
        upper = np.concatenate([idx[k * M:(k + 1) * M, k2 * M:(k2 + 1) * M].ravel()
                                for k in range(K) for k2 in range(k, K)])
        np.testing.assert_array_equal(np.sort(upper), np.arange(size))
        c = m // 2
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
