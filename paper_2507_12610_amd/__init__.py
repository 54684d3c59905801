"""Soft-sphere DEM hot path (TinyDEM, arXiv 2507.12610) on AMD MI355X.

The product is the C ABI in ``include/sdem.h`` implemented by HIP kernels in
``csrc/`` (built into ``libsdem.so``); ``sdem`` is its Python binding.
"""
from .sdem import (SDEM_FP64, SDEM_MIXED, Config, Params, SdemError, Solver,  # noqa: F401
                   autotune, copy_probe, lib, selftest_rounding)
