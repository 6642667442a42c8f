"""Plain, slow FP64 CPU oracle for Holographic Radiance Cascades (HRC).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.  The
product path (the HIP library and its Python binding) never imports it, and it
never imports the product path: the two share no code, tables or constants.

Modules
-------
``hrc``         forward pass: interval algebra (Eq. 5-9), seeded traces,
                merge up (Eq. 18-20), merge down (Eq. 13-17), quadrant gather
                (Algorithm 1 ``Lighting``).
``hrc_vjp``     the hand-written reverse pass of ``hrc`` (vector-Jacobian product).
``blur``        the cross blur after Algorithm 1 (Eq. 21, opacity rejection) and
                its adjoint.
``multibounce`` several diffuse bounces (fluence fed back as an in-scattering
                source, Section 4.2) and their reverse pass.
``bruteforce``  direct many-direction ray march of Eq. 1-3 (C, OpenMP) for the
                method's approximation error.
``closed_forms`` closed-form fluences that pin the brute force.
"""
