"""CPU oracle for exact k-NN Euclidean search with iSAX summaries.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls, links
or executes anything in this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark do.  It shares no code with the HIP library
(no kernels, headers, helpers, tables or constant generators).

Modules
  isax_ref   PAA, breakpoints, iSAX symbols, interleaved keys, leaf layout,
             mindist lower bounds (numpy / scipy, FP64 unless stated)
  knn_ref    brute-force exact k-NN in FP64 (numpy), and a plain-C twin
             (knn_ref.c, built by build_c()) used for large sampled checks
             and for the CPU baseline timing
  margin_ref FP64 check of the BF16 / FP8 dot-product filter margin
  spectral_ref  DCT-based reduced copy of the filter and its lower bound
"""
from . import isax_ref, knn_ref, margin_ref, spectral_ref  # noqa: F401
