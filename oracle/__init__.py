"""CPU FP64 oracle for the matrix-free SEM / SEM-NI monodomain operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the library path imports, calls or
links this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code, tables or constants with the HIP library
(the seeded input generators in `synth` are the one common module, and they
hold no arithmetic of the method).

What it computes, and from where in the paper (arXiv 2205.05136):
  quadrature.py  LG and LGL rules (Section 3, SEM and SEM-NI paragraphs)
  basis.py       nodal Lagrange bases on LGL nodes, dense 3D tensor arrays (Section 3)
  mesh.py        structured Q_p hexahedral lattices, shear and fiber recipe
  operator.py    explicit element matrices M_e, K_e(sigma) with the diffusion
                 tensor of Section 2 and A = alpha*M + K (Section 3, the linear
                 system); assembled CSR (Alg. 2, matrix-based) and dense
                 element action (Alg. 1's cell loop without sum factorisation)
  solvers.py     CG/PCG/FCG (Section 4), Lanczos lambda_max from CG
                 coefficients, Chebyshev-Jacobi smoother and V-cycle
                 (Sections 4.3 and 5), fast diagonalisation (textbook)
  multigrid.py   p- and octree h-prolongation as explicit sparse matrices (Section 4.3)
  adjoint.py     dL/dsigma per element through the solve (not in the paper)
  ionic.py       Aliev-Panfilov IMEX and BDF2 steps and pointwise RHS (stand-in
                 for the paper's cited ionic models; parity unpinned against
                 paper values), activation times as the time of the largest
                 |dV/dt| (Section 5.1)

Every function is plain and slow on purpose: element matrices are dense
(P^3 x P^3) and nothing is sum-factorised, blocked or fused.
"""
