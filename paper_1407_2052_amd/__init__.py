"""MI355X-native conservative finite-difference MP5 / Lax-Friedrichs / SSPRK
hot path (Porth et al. 2014, Sect. 2) behind a C-ABI library.

The native library is loaded lazily by :mod:`paper_1407_2052_amd.amrvac`; this
package import itself touches no GPU.
"""
__all__ = ["inputs"]
