"""CPU FP64 oracle for the block-preconditioned VIE-FFT solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports or calls this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may use it.  It shares no code with the HIP library.

It is a plain, slow, obviously-correct restatement of the method of Huang &
Sha, "A Parallel Block Preconditioner Based VIE-FFT Algorithm for Modeling
Electromagnetic Response from Nanostructures" (arXiv 2501.13512):

* ``green``    the discretised dyadic Green's tensor T(m) (eq. (1), with the
               scalar Green's function defined after it) and its circulant
               embedding (Sec. I: Toeplitz structure, FFT);
* ``operator`` the VIE operator of eqs. (2)-(4)/(6): dense assembly, a
               brute-force O(N^2) product and the FFT product;
* ``krylov``   BiCGSTAB with the right block-diagonal preconditioner of
               Sec. II-B (eqs. (10)-(11)), a dense LU reference solve, and
               the mixed-precision mode (complex64 products, FP64 vectors,
               FP64 residual and correction solves);
* ``physics``  plane-wave excitation, power balance, far field and RCS, and
               the Mie series used in Sec. III.

Unknown: P = J / (j omega eps0) (same Krylov iterates as the paper's J up to
the constant factor), so the operator is dimensionless:

    P_m / chi_m - sum_{n in S} T(m - n) P_n = E_inc(r_m),   m in S,

with chi = eps_r - 1 and S the non-vacuum voxels; E_tot = P / chi (eq. (2)).

Every function cites the passage it follows.  Parity status of each part is
listed in ``tests/`` next to its pins.
"""
