"""CPU FP64 oracle for the optimized Schwarz method (test infrastructure only).

This package is a plain, slow, deliberately unoptimised reference written from
the paper: the gravity Poisson problem of Sec. 2, its Q2 finite-element
discretisation, a global direct solve, and the non-overlapping Schwarz
iteration with Robin transmission conditions of Sec. 3 using exact subdomain
solves. It shares no code with the HIP library. Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never does.

Modules
  fe         Q2 Lagrange basis, Gauss quadrature, element matrices
  mesh       box mesh, node/element numbering, Dirichlet nodes
  assemble   global stiffness and load by element loops
  partition  box partitions, subdomain closures, directed interface faces
  subdomain  Robin-augmented subdomain matrices and face mass matrices
  direct     sparse LU and fast-diagonalisation direct solvers
  schwarz    the Jacobi Robin-Schwarz iteration with exact subdomain solves
  fourier    closed-form two-subdomain contraction factors
"""
