"""CPU oracle for tensorial template matching (TTM) -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 numpy implementation of what the TTM hot path computes,
written from the paper (Martinez-Sanchez et al., "Tensorial template matching
for fast cross-correlation with rotations and its application for tomography",
arXiv 2408.02398).  Correlations are direct spatial sums (the definition of
cross-correlation, Eq. "correlation"), not FFTs.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product (the HIP library and its Python binding)
never imports, calls or links it, and it never imports the product.

Modules
-------
sym        symmetric-tensor index set, multinomial weights, monomials,
           contractions, full-tensor expansion, sphere moments
rotations  quaternion algebra, the cube group, trilinear pull-back rotation
ttm        filter, template normalisation (Eq. norm_t), tensor template
           (Eq. tt / Alg. 1), local normalisation (Eq. norm_f), tensor field
           (Eq. tcc / Alg. 2), Frobenius score, SS-HOPM orientation, peaks,
           brute-force rotation-sampled TM (Eq. lncc)
mlp        FP64 reference of the learned-start network (forward, backward, Adam)

Parity status of each function is stated in its module header.
"""
