"""CPU FP64 oracle for singular value thresholding (SVT) matrix completion.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library: the only module both sides use is ``workload``, which draws inputs.

Contents (each function cites the passage of the paper it writes out):

* ``jacobi_svd``       dense full SVD by one-sided Jacobi (C, ``jacobi.c``)
* ``shrink``           the singular value shrinkage operator D_tau, eq. (2.2)
* ``top_triplets_dense`` the largest singular triplets of a dense matrix
* ``k0_kick``          the number of skipped initial steps, eq. (5.3)
* ``apply_sparse``     Y x and Y^T x for Y supported on Omega (Section 2.2)
* ``sampled_entries``  X_ij = sum_l U_il V_jl on Omega
* ``svt_dense``        Algorithm 1 (Section 5.1.5), tier A: dense Y, full SVD
* ``svt_continuation`` tau continuation with warm starts (Section 6)
* ``gram_triplets``    singular triplets above tau of a sparse Y from its Gram
                       matrix's eigendecomposition (LAPACK, FP64)
* ``svt_sparse``       Algorithm 1, tier B: sparse Y, Gram-matrix triplets
* ``krylov.svt_krylov`` Algorithm 1, tier C: sparse Y, the s_k largest
                       triplets from a library partial SVD (SciPy / ARPACK),
                       the repeat loop over s_k as printed

Modules beside the package's exports: ``general`` (linear measurements,
Section 3.1), ``dantzig`` (the matrix Dantzig selector, Section 3.3),
``randomized`` (the randomised partial SVD, Section 6), ``block_krylov``
(block bidiagonalisation, an experiment) and ``partial_reorth``
(bidiagonalisation with partial reorthogonalisation, Section 5.1.1).
"""
from .svt import (  # noqa: F401
    jacobi_svd,
    shrink,
    k0_kick,
    apply_sparse,
    sampled_entries,
    svt_dense,
    svt_continuation,
    top_triplets_dense,
    gram_triplets,
    svt_sparse,
)
