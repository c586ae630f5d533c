"""Heated simulated bifurcation (Kanao & Goto, arXiv:2203.08361) on AMD MI355X.

The computation lives in the HIP library libhsb.so (C ABI in include/hsb.h);
`hsb` is its Python binding and `metrics` holds the evaluation quantities of
the paper (cut value, step-to-solution).
"""
from . import hsb, metrics  # noqa: F401
from .hsb import Context  # noqa: F401
