"""FP64 CPU reference implementation ("the oracle") of the primal-dual
symmetric-cone MWU method of Zheng, Varvitsiotis, Tan and Lin,
"A Primal-Dual Framework for Symmetric Cone Programming" (arXiv 2405.09157).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link this package; only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use it.
It shares no code, table or helper with the GPU path.

Modules
-------
eja      Euclidean Jordan algebra of the second-order cone and the orthant:
         Jordan product, spectral decomposition, trace, Loewner exponential
         (Section 2.1).
scmwu    The SCMWU online learner over product cones (Section 2.3, eq. SCMWU),
         including a product of an orthant and Lorentz blocks of mixed sizes.
ses      Smallest enclosing sphere via the max-form meta-algorithm
         (Section 3 with Section 4.1): alpha-FTP loop, closed-form ORACLE,
         monitor f(t), early stopping (Section 5), adaptive alpha search.
svm      Hard-margin SVM / polytope distance via the min-form meta-algorithm
         (Section 3 "Extension to minimization problems" with Section 4.2).
ses_grad Gradient of the radius after a fixed number of SES iterations by
         the adjoint recursion (reverse pass through the unrolled iterations).
exact    Exact references used to pin the above: Welzl's algorithm and brute
         force for SES, direction enumeration for 2-D SVM.
certify  Certified bounds for any candidate (upper/lower bounds on OPT).

Every number is IEEE binary64.  Pinning status of each function is stated in
its module header.
"""
