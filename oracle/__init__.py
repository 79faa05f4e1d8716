"""Plain FP64 CPU oracle of HNTL search (test infrastructure).

This package is test infrastructure.  Only ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark may import it; the GPU library never does,
and the oracle imports nothing from the GPU library.  The two share only the
seeded input generators in ``workloads/``.

Every function follows the paper's description step by step in float64 (numpy,
with LAPACK ``eigh`` and BLAS matmul as library primitives), without blocking,
fusion or reordering beyond what the definition states:

* ``kmeans``   grain partitioning (k-means++ seeding, Lloyd iterations)
* ``pca``      per-grain local PCA basis (Section 2.2)
* ``index``    codes and residual energies, eq. (1)-(4)
* ``search``   routing (Section 2.1 step 1, Section 2.3), projection
               (eq. 1-4), tangent scan score (eq. 6), top-C pool, exact rerank
               (Section 2.1, Mode B)
* ``brute``    exact k-nearest neighbours (ground truth)
* ``router``   MLP router forward/backward, softmax cross-entropy, Adam
* ``quant``    BF16 / FP8-e4m3 rounding emulation for the precision form

Parity status of each function is stated in its module header.
"""
from . import brute, index, kmeans, pca, search  # noqa: F401
