"""Reference oracle for the ChFSI hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 CPU implementation (numpy/scipy) of what the GPU library
computes, written from the paper's description of the spectral finite-element
Kohn-Sham eigenproblem (Sec. 2.4, eq. hep), of Chebyshev-filtered subspace
iteration (Sec. 3.3 eq. chebFilter, Sec. 3.4 Alg. 3 CholGS, Sec. 3.5 RR) and
of the electron density (Sec. 3.5, Alg. 5).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_1903_10959_amd``) and imports nothing from it; the only module both
sides use is the seeded input generator ``workload``.

Modules
-------
``fem``    GLL rule, Lagrange derivative matrix, cell matrices, numbering,
           colouring, CSR assembly of the standard-form Hamiltonian and its
           Kronecker-sum form (Sec. 2.4).
``chfsi``  Chebyshev filter (paper's unscaled recursion and the normalised
           one), CholGS (FP64 and the paper's mixed variant), Rayleigh-Ritz,
           the subspace-iteration loop, dense and Lanczos eigensolves.
``density`` Spectrum-splitting Rayleigh-Ritz (Alg. 4), Fermi-Dirac occupancy
           and Fermi level, the nodal electron density by eq. elecDensSP and
           by eq. elecDens, and the cell-level form of eq. elecDensSums
           (Sec. 3.5, Alg. 5).
``kpoint`` The periodic Bloch operator at a k-point (Sec. 2.1 eq.
           ksproblemPer): periodic numbering, the GLL first-derivative cell
           matrices, the complex Hermitian standard-form CSR and its
           Kronecker-sum apply.
``poisson`` The discrete Poisson problem of the electrostatics (Sec. 2.4 eq.
           phiTotDiscreteSolve, Dirichlet) and the Jacobi-preconditioned
           conjugate-gradient solver the paper uses for it.

Pinning status (what each function is checked against) is listed in the
module docstrings.  The paper's mixed-precision steps (CholGS, the projected
Hamiltonian) are pinned by exactly rounded sums and FP32 error bounds; the
reduced-precision filters are not the paper's and have no oracle of their
own: their results are measured against the FP64 functions here.
"""
