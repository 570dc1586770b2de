"""MI355X-native sample-based quantum diagonalization hot path.

The compiled library ``libsqd.so`` (HIP kernels behind a C ABI) is loaded on
first use by :mod:`paper_2601_16169_amd.sqd`; importing this package alone
loads nothing.
"""
__all__ = ["inputs"]
