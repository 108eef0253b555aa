"""Pin of the Philox oracle: published known-answer vectors, the normals they
give through Box-Muller, and the law and independence of the normals."""
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


def test_first_normal_from_the_known_answer_words():
    # seed 0, stream 0, element 0 uses counter (0, 0, 0, 0) and key (0, 0),
    # whose published output words 0 and 1 give the Box-Muller pair
    u0 = (0x6627E8D5 + 1) / 2.0 ** 32
    u1 = (0xE169C58D + 1) / 2.0 ** 32
    z0 = np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)
    assert philox.normals(0, 0, 1)[0] == z0


def test_normals_follow_the_standard_normal_law():
    # Kolmogorov-Smirnov against the standard normal CDF, the tail mass beyond
    # 3 sigma, and no correlation between neighbours or between streams
    from scipy import stats
    z = philox.normals(2024, 3, 100000)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(np.mean(np.abs(z) > 3.0) - 2 * stats.norm.sf(3.0)) < 6e-4
    assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 0.01
    assert abs(np.corrcoef(z, philox.normals(2024, 4, 100000))[0, 1]) < 0.01
