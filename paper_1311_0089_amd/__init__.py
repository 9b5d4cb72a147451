"""MI355X-native FFT-Galerkin homogenization (Vondrejc, Zeman & Marek).

The compute path is the HIP library ``libhom.so`` (hand-written gfx950
kernels behind the C ABI of ``include/hom.h``); this package is a thin ctypes
binding over it.  Importing the package does not load the library; the first
use does, and fails loudly if it has not been built.
"""
from .hom import (Cell, HomError, Server, lib, GANI, GA, FP64, MIXED, ISO, DIAG, FULLSYM, ELASTIC,
                  EXPORTED_SYMBOLS, set_specialized, tune_save, tune_load)

__all__ = ["Cell", "Server", "HomError", "lib", "GANI", "GA", "FP64", "MIXED", "ISO", "DIAG",
           "FULLSYM", "EXPORTED_SYMBOLS", "set_specialized", "tune_save", "tune_load"]
