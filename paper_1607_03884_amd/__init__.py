"""Batched constant-pressure Radau IIA chemical-kinetics integration on MI355X.

The HIP library (librkchem.so, C ABI in include/rkchem.h) does all the work;
`Mechanism` is its thin Python binding over PyTorch device tensors.
"""
from ._lib import Mechanism, RkError, RkStats, LIB_PATH  # noqa: F401
