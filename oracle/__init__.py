"""CPU FP64 oracle for the SAP-preconditioned FGMRES-DR Wilson-Dirac solver.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
NumPy/SciPy restatement of what the paper (Frommer, Nobile, Zingler,
"Deflation and Flexible SAP-Preconditioning of GMRES in Lattice QCD
Simulation", arXiv:1204.5463) computes. It exists to check the HIP
implementation; only the tests, the smoke check and the benchmark's CPU
baseline may import it. The product library never calls into it and shares
no code with it.

Modules:
  wilson    -- the Wilson-Dirac operator (eq. 1) and its block restriction
               (eq. 2), dense assembly for brute-force checks (Section 2).
  sap       -- minimal-residual block solves, the SAP sweep (Alg. 2), the
               sequential multiplicative Schwarz (Alg. 1) and the truncated
               series M_s of the block splitting (Section 4).
  fgmresdr  -- the flexible Arnoldi process (Alg. 3) and FGMRES-DR
               (Alg. 4) with the explicit-residual / clean-restart policy
               (Section 4.7).
"""
