"""FP64 CPU oracle for GleanVec / LeanVec-Sphering (test infrastructure only).

This package is the *checker*: a plain, slow, obviously correct NumPy
implementation of what the search path computes, written from the paper
(GleanVec, arXiv 2410.22347).  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product library never
does, and it shares no code with the HIP path.

Modules
-------
formats   -- round-to-nearest-even converters to FP16 / BF16 / FP8-E4M3FN
rng       -- SplitMix64 (published definition) and the fit's sampling draws
gleanvec  -- spherical k-means, second moments, sphering fit, encode,
             eager projection, reduced scoring, exact top-k, rerank,
             ground truth, loss and gradient (pairwise and Gram forms)

Parity status: every function is pinned by tests under ``tests/``
(``-m "not gpu"``) against closed forms, invariants, textbook special cases
or brute force.  The only unpinned part is global optimality of k-means
(a local method): "parity unpinned" for that property alone.
"""
from . import formats, rng, gleanvec  # noqa: F401
