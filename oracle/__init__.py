"""CPU oracle for the Ozaki-I FP64 / complex-FP64 GEMM emulation.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
reference. Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it. The GPU library never imports, links or calls anything here,
and nothing here imports the GPU library: the two share no code. The only common
module is ``workloads`` (seeded random inputs, no emulation arithmetic).

Contents
--------
ozaki    the emulation model itself: exponents, trunc-7 split, exact slice-pair
         products, FP64 recombination, alpha/beta (Section 2.2).
dd       double-double GEMM, the accuracy reference (Hida, Li and Bailey 2001,
         cited in Section 2.2).
exact    exact rational entries of op(A) op(B) with Python integers.
metrics  componentwise, normwise and elementwise error measures.

What the paper fixes and what is read into it is listed in the module
docstring of ``oracle.ozaki``.
"""
