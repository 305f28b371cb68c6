"""CPU FP64 oracle for the controllability method (CMCG) for the Helmholtz equation.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct reference
that the GPU path is checked against.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product (the HIP library and its Python
binding) never does, and shares no code with it.

Modules
-------
* ``f1``    first-order (velocity / flux) staggered leapfrog scheme, its literal transpose,
            the energy metric, the filter and the frequency-domain system (Sec. 3, eq. mixWE,
            eq. mix_cost_functional_J, eq. mixJ_deriative_2, eq. TH_FILTERED_MIXED_SOLUTION).
* ``f2``    second-order nodal leapfrog scheme with lumped mass, its literal transpose, the
            energy metric, the Riesz map and the filter (Sec. 2, eq. WE, eq.
            cost_functional_J, eq. CMCG_PRECONDITIONIER, eq. fundamental-frequency-solution).
* ``cmcg``  the CMCG Algorithm of Sec. 2.3 (Steps 1-6), written once for any scheme that
            supplies the period maps, the metric and the Riesz map.

Pins (tests/test_oracle_*.py) tie every function to something other than itself:
closed-form leapfrog dispersion, discrete energy conservation, the damped energy identity,
brute-force dense transposes, the direct sparse solve of the time-discretised Helmholtz
system, CG monotonicity, filter invariances, symmetry, reciprocity and the paper's 1D
closed-form solutions in channel form.
"""
