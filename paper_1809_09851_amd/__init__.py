"""MI355X-native evaluation of the FDBB compressible-Euler building blocks.

The hot path lives in the HIP library ``libfdbb.so`` (``csrc/``); the
Python modules here only marshal arguments into its C ABI.
"""
