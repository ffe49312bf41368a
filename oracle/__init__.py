"""CPU float64 oracle for the sum-of-Kronecker-plus-diagonal solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU library: it is
plain numpy/scipy in float64, written from the paper (CoLA, arxiv 2309.03060)
so a reader can check each function against the passage it cites.

Modules
-------
kron     operator definition, dense materialisation, structured MVM
         (Sec. 3.1 base operators, Sec. 3.2 Sum/Kronecker composition, Table 2)
direct   exact solves: dense Cholesky; Kronecker eigendecomposition
         (App. A "Eigendecomposition" and "Derived functions")
cg       textbook conjugate gradients (the PSD base case of App. C, Table
         "iterative methods") and float64-residual iterative refinement
grad     solve VJP (App. B.2, autograd rule 1) by three routes: dense
         -lambda x^T contraction, closed-form factor contractions, finite
         differences
lowprec  bf16 / fp32 rounding emulator (diagnostic; App. C.3 context)
slq      log det by stochastic Lanczos quadrature with the tridiagonal taken
         from CG coefficients, Kronecker closed forms of log det and
         Tr(A^{-1}) (App. A "Derived functions"; App. C base-case table)
precond  preconditioned CG (Jacobi from the exact Kronecker diagonal rule,
         Kronecker-eigen of the first term), Hutchinson and doubly
         stochastic diagonal estimators with their per-entry variances
         (App. A "Diagonal"; Sec. 3.3; App. B.1)

Conventions: vec is row-major (C order), so (K1 (x) K2) x = vec(K1 X K2^T)
with X = x.reshape(n1, n2), matching numpy.kron and the row-major form of the
Kronecker-diagonal rule of App. A.  Right-hand sides are rows: B has shape
(nrhs, n).

Parity status of each function is stated in its docstring; every function
here is pinned by tests in tests/test_oracle_*.py.  The two mixed-precision
schedules (restarted refinement, reliable updates) are readings: the paper
gives no low-precision CG steps, so their pins are what mathematics fixes
(textbook CG when nothing is rounded, float64 accuracy from float32 vectors,
a bound on the number of residual replacements, stagnation under an
inconsistent inner operator), not printed values.
"""
from . import kron, direct, cg, grad, lowprec  # noqa: F401
