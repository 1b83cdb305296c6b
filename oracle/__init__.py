"""CPU oracle for polynomial RS(k,m) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It wraps the plain C implementation in rs_oracle.c with ctypes
and numpy; it shares no code with the GPU library.
"""
from .oracle import (Field, genpoly, encode, decode, syndromes, vandermonde,
                     invert, position, load)

__all__ = ["Field", "genpoly", "encode", "decode", "syndromes", "vandermonde",
           "invert", "position", "load"]
