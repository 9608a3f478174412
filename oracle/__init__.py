"""CPU FP64 oracle for the explicit OTM step (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it: the only common module is the seeded input generator,
which holds no arithmetic of the method.

The oracle follows the paper (Kumar, Gosselet, Huang, Weissenfels, Wriggers,
"Parallel multiphysics simulation for the stabilized optimal transportation
meshfree (OTM) method"):

* ``search``   -- support domains (Sec. 3, linked-cell scheme of Alg. 3) and
                  their brute-force definition;
* ``lme``      -- local max-ent shape functions (Sec. 2.3, LME equation) and
                  their spatial gradient;
* ``material`` -- Neo-Hookean stress, finite-strain J2 with Hencky strain and
                  exponential map (Sec. 4.1), Johnson-Cook flow stress and
                  adiabatic heating (Sec. 4.2);
* ``step``     -- the explicit step of Alg. 1: lumped mass and nodal force,
                  central difference and wall contact, MP position and
                  deformation gradient, constitutive update, search, shape
                  functions.

Every function is plain NumPy in float64 (complex128 where a complex-step
derivative is taken), vectorised over material points, with no blocking or
reordering beyond what the definitions state.
"""
