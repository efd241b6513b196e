"""The binary32 coordinate of a grid point rebuilt from its int8 copy: the binary64 product
k * (1/255) rounded to binary32 equals the correctly rounded binary32 quotient k / 255 for
every k in [0, 255], so projections read from the int8 copy see the values X holds."""

import numpy as np


def test_grid_coordinate_formula_is_the_correctly_rounded_quotient():
    k = np.arange(256)
    quotient = k.astype(np.float32) / np.float32(255)  # IEEE binary32 division, correctly rounded
    rebuilt = (k.astype(np.float64) * (1.0 / 255.0)).astype(np.float32)
    np.testing.assert_array_equal(rebuilt.view(np.uint32), quotient.view(np.uint32))
    # the single-precision product is not: the formula needs the binary64 step
    assert (k.astype(np.float32) * np.float32(1.0 / 255.0) != quotient).any()


def test_int8_copy_round_trip():
    # the stored byte is k - 128; flipping the top bit of each byte gives k back
    k = np.arange(256, dtype=np.int64)
    stored = (k - 128).astype(np.int8)
    word = stored.view(np.uint8).astype(np.uint32) ^ 0x80
    np.testing.assert_array_equal(word, k)
