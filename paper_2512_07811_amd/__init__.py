"""qtthom: MI355X-native hot path of SFFT/QTT Lippmann-Schwinger homogenization.

The package is deliberately light at import time: the HIP library is loaded
on first use by :mod:`paper_2512_07811_amd.qtt`, and the seeded input
generators in :mod:`paper_2512_07811_amd.inputs` import nothing but numpy.
"""

__all__ = ["inputs"]
