"""CPU oracle for the coarse-grid-projection hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, fp64 implementation of what the HIP library computes, written
from the paper (Kashefi, "A coarse-grid projection method for accelerating
incompressible MHD flow simulations", arXiv 2003.00082):

* ``oracle.mesh``   nested 4-way refinement (Section 2.3, Eq. 18), injection
                    (Eq. 19) and P1 prolongation (Eq. 20);
* ``oracle.fem``    Galerkin P1 stiffness (Section 2.3), the coarse sources of
                    Eqs. 12 and 15, the Lorentz-force source of Eqs. 13-14 and
                    the velocity correction of Eqs. 16-17;
* ``oracle.solve``  the exact coarse solution (sparse/dense direct factorisation)
                    and Jacobi-preconditioned CG in fp64 and in fp32 with fp64
                    iterative refinement (plain C, ``oracle/pcg_oracle.c``),
                    with the Jacobi or a Chebyshev polynomial preconditioner;
* ``oracle.deflation``  subdomain-deflated PCG (an extension: aggregates from
                    recursive coordinate bisection, Nicolaides / Saad et al.);
* ``oracle.gnn``    the learned initial-guess network, forward and analytic
                    backward in fp64 with bf16 rounding emulated;
* ``oracle.momentum``  the semi-implicit momentum step of Eqs. 13-14 on the fine
                    mesh (P1 mass, convection and viscous operators, direct solve);
* ``oracle.locate`` P1 interpolation at arbitrary points by brute-force point
                    location (the general, non-nested restriction of Section 2.3).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.
"""
