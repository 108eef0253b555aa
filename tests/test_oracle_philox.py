"""Pin of the Philox oracle: published known-answer vectors and moments."""
import numpy as np

from oracle import philox


def test_known_answer_vectors():
    # Random123 kat_vectors for philox4x32_10: counter, key -> output
    out = philox.philox4x32_10([0], [0], [0], [0], 0, 0)
    assert [int(x[0]) for x in out] == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    out = philox.philox4x32_10([0xFFFFFFFF], [0xFFFFFFFF], [0xFFFFFFFF], [0xFFFFFFFF],
                               0xFFFFFFFF, 0xFFFFFFFF)
    assert [int(x[0]) for x in out] == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    out = philox.philox4x32_10([0x243F6A88], [0x85A308D3], [0x13198A2E], [0x03707344],
                               0xA4093822, 0x299F31D0)
    assert [int(x[0]) for x in out] == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_normal_moments():
    z = philox.normals(12345, 7, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
