"""The host reference of the device normal generator, pinned to the
published known-answer vectors of Philox4x32-10 (Random123, Salmon et al.,
SC11) and to the first moments of N(0, 1)."""
import numpy as np

from philox_ref import normals, philox4x32_10


def test_philox_known_answers():
    assert philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                         [0xA4093822, 0x299F31D0]) == [0xD16CFE09, 0x94FDCCEB, 0x5001E420,
                                                       0x24126EA1]


def test_normal_moments_and_offsets():
    x = normals(12345, 0, 20000)
    assert abs(x.mean()) < 4 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / x.size)
    assert abs(np.mean(x ** 4) - 3.0) < 0.15
    # a window of the stream is the stream
    np.testing.assert_array_equal(normals(12345, 777, 50), x[777:827])
