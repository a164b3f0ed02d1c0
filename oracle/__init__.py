"""FP64 CPU oracle for the Blahut-Arimoto iteration on the finite-length binary
deletion channel BDC_d (Pinto & Ribeiro, "Improved Capacity Upper Bounds for the
Deletion Channel using a Parallelized Blahut-Arimoto Algorithm").

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or runs
anything here.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use this package.

Contents
--------
``oracle.bdc``     plain numpy implementation: brute-force embedding counts over
                   position subsets, the dense channel matrix, the BA iteration
                   in the order of Section 2.3, the Blahut bounds, the mutual
                   information and its closed-form gradients.
``oracle.native``  ctypes loader for ``oracle/c/bdc_oracle.c`` (plain C with
                   OpenMP): brute-force rows for any n <= 24, a CSR channel for
                   n <= 16 with an FP64 BA on it, and the product-distribution
                   closed forms used for sampled checks at n = 20.

The oracle shares no code with the HIP path.
"""
