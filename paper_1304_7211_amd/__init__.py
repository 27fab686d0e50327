"""MI355X-native Richardson-Lucy deconvolution (hot path in HIP, C ABI in include/rl.h).

Python side: ``_abi`` (ctypes marshalling of every C entry point, same names) and
``job`` (torch tensors as the memory and stream provider).  The library ``librl.so`` is
built in-tree by ``paper_1304_7211_amd.build``; importing ``_abi`` functions raises if it
is missing -- there is no CPU fallback.
"""
from . import _abi
from ._abi import (RLError, rl_active_list, rl_batch_workspace_bytes, rl_destroy,
                   rl_get_state, rl_init, rl_iterate, rl_iterate_batch, rl_job_describe,
                   rl_psf_runs, rl_result, rl_set_state, rl_thin_schedule, rl_timing_enable,
                   rl_timing_read, rl_timing_reset, rl_workspace_bytes)

__all__ = ["_abi", "RLError", "rl_active_list", "rl_batch_workspace_bytes", "rl_destroy",
           "rl_get_state", "rl_init", "rl_iterate", "rl_iterate_batch", "rl_job_describe",
           "rl_psf_runs", "rl_result", "rl_set_state", "rl_thin_schedule", "rl_timing_enable",
           "rl_timing_read", "rl_timing_reset", "rl_workspace_bytes"]
