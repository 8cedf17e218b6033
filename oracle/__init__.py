"""CPU oracle for the BDDC hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy/SciPy implementation of what the hot path computes
(static condensation onto the interface, the BDDC preconditioner with deluxe
or counting scaling, the adaptive face eigenproblems, PCG with a Lanczos
condition estimate, interior recovery).  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path never calls it.  It shares no code with the HIP library: both consume
the same plain-data workloads produced by the ``inputs`` generator.

Every routine follows the paper's definitions step by step (citations in
the docstrings); algorithmic choices are deliberately different from the
library's (sparse LU with pivoting instead of a signed dense factorisation,
SVD instead of Gram-eigen + Householder, bordered LU instead of a
regularised inverse) so that agreement is evidence, not a tautology.
"""
