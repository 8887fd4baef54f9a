"""Batched algorithmic Matsubara integration (AMI) on MI355X (gfx950).

Python face of ``libamigpu.so`` (C ABI declared in ``include/amigpu.h``): a
thin ctypes layer that only marshals arguments.  Construction of the symbolic
solution (Burke & LeBlanc, arXiv 2311.17189, Sec. 2.2) runs in the library's
C++ host code; every evaluation step runs in its HIP kernels.  PyTorch is used
only to hold device memory and to name the stream.

The library must have been built (``paper_2311_17189_amd.build.build()`` or
``__graft_entry__.build()``); the first call into it raises ImportError
otherwise (there is no fallback path).
"""
from ._lib import (VARIANT_AUTO, VARIANT_PACKED, VARIANT_SPECIALIZED,  # noqa: F401
                   VARIANT_TABLES, VARIANT_TWO_PASS, AmiError, Batch, Terms, batch_source, evaluate, evaluate_adjoint,
                   evaluate_complex, evaluate_complex_adjoint, evaluate_hubbard, evaluate_hubbard_adjoint, evaluate_hubbard_adjoint_no_alloc,
                   integrate_hubbard, kernel_timer_start,
                   kernel_timer_stop, last_variant, lib_path, load_library, mc_estimate, measure_fp64_peak,
                   read_graph, set_two_pass_chunk_bytes, version)

__all__ = ["VARIANT_AUTO", "VARIANT_PACKED", "VARIANT_SPECIALIZED", "VARIANT_TABLES", "VARIANT_TWO_PASS", "AmiError", "Batch", "Terms", "batch_source", "evaluate", "evaluate_adjoint", "evaluate_complex", "evaluate_complex_adjoint", "evaluate_hubbard",
           "evaluate_hubbard_adjoint", "evaluate_hubbard_adjoint_no_alloc", "integrate_hubbard", "mc_estimate", "read_graph", "kernel_timer_start", "kernel_timer_stop", "measure_fp64_peak", "last_variant", "lib_path", "load_library", "set_two_pass_chunk_bytes",
           "version"]
