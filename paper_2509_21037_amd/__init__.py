"""Sparsity-aware assembly of FETI dual Schur complements on AMD MI355X.

The product path is libscasm.so (host planner + HIP kernels for gfx950) behind
the C ABI of include/scasm.h; `scasm` is its ctypes binding.
"""
from .scasm import (Plan, check_dual_tensor, host_analyze, host_tile_visits, autotune, autotune_classes, ScasmError, load, LIB_PATH, SC_OK, SC_ERR_INVALID_ARG, SC_ERR_NOT_SPD,
                    SC_ERR_OOM, SC_ERR_DEVICE, SC_ERR_UNSUPPORTED, SC_ERR_STATE, EXPORTED)

__all__ = ["Plan", "check_dual_tensor", "host_analyze", "host_tile_visits", "autotune", "autotune_classes", "ScasmError", "load", "LIB_PATH", "SC_OK", "SC_ERR_INVALID_ARG", "SC_ERR_NOT_SPD",
           "SC_ERR_OOM", "SC_ERR_DEVICE", "SC_ERR_UNSUPPORTED", "SC_ERR_STATE", "EXPORTED"]
