"""MI355X-native hybrid-PIC step of Morris, Robinson & Ridgers (arXiv 2107.01723).

The physics runs in HIP kernels behind the C ABI of include/hyb.h
(libhyb.so, built with `python -m paper_2107_01723_amd.build`); this package
is the thin Python binding (`Run`, `Engine`) and the serving driver.
"""
from .hyb import (FP32_MIXED, FP64, MODEL_KEYS, Engine, HybError, Run, check_abi,  # noqa: F401
                  footprint, lib, model_scan)
