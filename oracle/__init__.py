"""Plain FP64 CPU oracle for cascaded bilateral sampling (CABS).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path (the C-ABI library and its Python binding) never does, and it
shares no code, tables or constants with that path.

Contents
  philox.py    counter-based generator (Philox-4x64-10, Salmon et al., SC'11)
               and Floyd's sampling without replacement
  matrices.py  entry access to A (dense, low-rank + noise, RBF kernel)
  cabs.py      the method: pilot sampling, the sketching routine, the optional
               orthogonalisation, the weighted k-means follow-up sampling with
               snapping to in-sample points, the follow-up sketch, and the
               relative Frobenius error

Every floating-point step runs in float64 with NumPy/SciPy library primitives
(SVD, matrix product, pairwise squared distances), in the order the paper
gives.  Where the paper leaves a choice open, the reading taken is stated in
the docstring of the function that makes it.

Parity status: every function here is pinned by a CPU test against a closed
form, a library routine, a brute-force computation or an invariant; the one
exception is the paper's empirical claim that the follow-up sketch beats the
pilot sketch, which is not a property of the algorithm and is not tested.
"""
