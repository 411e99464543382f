"""MI355X (gfx950) implementation of MARS: multi-sample allocation through
Russian roulette and splitting (Meyer et al., SIGGRAPH Asia 2024).

The hot path is a HIP library (libmars.so) behind the C ABI declared in
include/mars.h; this package holds the ctypes binding (_capi) and a small
numpy/PyTorch front end (api)."""
from ._capi import MarsError, lib, mars_version  # noqa: F401
