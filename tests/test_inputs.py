"""The seeded input generator: determinism, normalisation and shapes."""

import numpy as np

import scsc_inputs as si


def test_field_deterministic_and_normalised():
    a = si.field(2, 3, 100, 100)
    b = si.field(2, 3, 100, 100)
    np.testing.assert_array_equal(a, b)
    assert abs(a.mean()) < 1e-12
    assert abs(a.std() - 1.0) < 1e-12
    assert not np.array_equal(a, si.field(2, 4, 100, 100))


def test_field_spectrum_decays():
    x = si.field(1, 0, 128, 128)
    P = np.abs(np.fft.fft2(x)) ** 2
    f = np.sqrt(np.fft.fftfreq(128)[:, None] ** 2 + np.fft.fftfreq(128)[None, :] ** 2)
    low = P[(f > 0.02) & (f < 0.05)].mean()
    high = P[(f > 0.3) & (f < 0.45)].mean()
    assert low > high


def test_filters_unit_norm():
    d = si.filters(1, 16, 11)
    assert d.shape == (16, 11, 11)
    np.testing.assert_allclose(np.sqrt((d ** 2).sum(axis=(1, 2))), 1.0, rtol=1e-14)


def test_ragged_sizes_range():
    s = si.ragged_sizes(4, 256)
    assert s.shape == (256, 2)
    assert s.min() >= 64 and s.max() <= 512
    np.testing.assert_array_equal(s, si.ragged_sizes(4, 256))


def test_field_default_is_the_sigma_2_normalisation():
    a = si.field(5, 1, 40, 30)
    np.testing.assert_array_equal(a, si.field(5, 1, 40, 30, lcn_sigma=2.0))
    raw = si.field(5, 1, 40, 30, lcn_sigma=None)
    assert abs(raw.mean()) < 1e-12 and abs(raw.std() - 1.0) < 1e-12
    assert not np.allclose(raw, a)
    np.testing.assert_array_equal(si.stream_batch(5, 2, 3, 40, 30, lcn_sigma=8.0)[1],
                                  si.field(5, 4, 40, 30, lcn_sigma=8.0))
