"""Plain, slow, FP64 reference implementation of directional H2 compression.

TEST INFRASTRUCTURE ONLY.  This package is the oracle that the GPU library is
checked against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the library itself never does, and this package
imports nothing from the library.  It follows S. Boerm, "Directional
H2-matrix compression for high-frequency problems" (2015):

* ``plan``     cluster tree, directions, son maps, block tree, column sets
               (Section 2 definitions, Section 3 admissibility, Section 6 sets)
* ``matrix``   matrix entries of the point-Nystroem Helmholtz single layer
* ``compress`` basis construction, coupling matrices, near field
               (Section 6, the basis algorithm and the error-control remark)
* ``dh2``      the DH2 representation, its matrix-vector product
               (Section 4) and the spectral error measure (Section 7)

Every numerical step is written from its definition, in float64/complex128,
with LAPACK SVDs from numpy as the only library primitive.  Nothing is
blocked, fused or reordered beyond what the definitions state.
"""
