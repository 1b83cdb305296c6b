"""MI355X-native polynomial Reed-Solomon RS(k,m) erasure coding.

The codec runs in hand-written HIP kernels behind the C ABI of
librs_poly.so (include/rs_poly.h); `binding` marshals arguments to it.
Importing the package loads nothing; the library is opened on first use.
"""

__all__ = ["binding", "build"]
