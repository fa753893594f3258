"""FP64 CPU oracle for the many-flavor blocked quark solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or execute anything in this package; only
the tests, the smoke check and the benchmark's CPU-baseline leg use it.

The oracle computes the plain definitions, on the full lattice (no even/odd
split), in numpy complex128:

* ``dirac``   -- Wilson-Dirac operator D = 1 - kappa H and its adjoint, each
                 coded from its own formula, with Schroedinger-functional,
                 periodic or time-antiperiodic boundaries (Section 2; Sec. 3.1).
* ``solvers`` -- per-RHS Hestenes-Stiefel CG on the normal equations and the
                 two solves of the blocked force algorithm (Alg. 1 and Alg. 2),
                 plus dense direct solves for tiny lattices.
* ``force``   -- the pseudo-fermion action sum_i |D^-1 phi_i|^2 (Eq. 2) and the
                 MD force summed over pseudo-fermions (Eq. 3), written as the
                 literal derivative per su(3) generator.
* ``schur``   -- the even/odd Schur complement D^ = 1 - kappa^2 H_eo H_oe,
                 solves of D and D^+ through it, and the even/odd action
                 variant S_eo = sum_i |D^-1 phi_i,e|^2 with its force.
* ``bicgstab``-- the paper's solver family on D: per-RHS BiCGStab, the global
                 (Gl-) and block (Bl-) BiCGStab of Sec. 3.1, each with an
                 optional right preconditioner (the mixed-precision inner
                 solve of Sec. 3.2).
* ``hmc``     -- leapfrog molecular dynamics and Delta-H for the dt^2 pin.
* ``ptc``     -- the gauge-covariant parallel-transport convolution network
                 used as a learned preconditioner, forward and adjoint.
* ``fgmres``  -- restarted flexible GMRES with right preconditioning.

Inputs come from the ``synth`` generators; the oracle shares no code with the
GPU path.
"""
