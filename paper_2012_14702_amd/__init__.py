"""MI355X (gfx950) Iterative Perturbation Theory eigensolver.

The compute lives in ``libipt.so`` (hand-written HIP kernels behind the C ABI of
``include/ipt.h``); ``paper_2012_14702_amd.ipt`` is a thin ctypes binding with the
same entry-point names.  PyTorch supplies device memory and the current stream.
"""
from .ipt import (CONVERGED, DIVERGED, MLP, NOT_CONVERGED, IPTError, Handle, Opts, ipt_batched_get_tiles,
                  ipt_batched_set_tiles, ipt_batched_tune, ipt_solve_batched, ipt_solve_csr, ipt_solve_dense,
                  library_path, load_library)

__all__ = ["CONVERGED", "NOT_CONVERGED", "DIVERGED", "IPTError", "Handle", "MLP", "Opts", "ipt_solve_dense",
           "ipt_solve_csr", "ipt_solve_batched", "ipt_batched_tune", "ipt_batched_get_tiles", "ipt_batched_set_tiles",
           "load_library", "library_path"]
