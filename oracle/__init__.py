"""Plain FP64 CPU oracle for one differentiable MAC-grid Navier-Stokes step.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct reference
that the GPU library is checked against.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the GPU library never
does, and the two share no code (only the seeded input generators in
``scenes``, which contain none of the method's arithmetic).

Everything is float64 numpy/scipy, written from the paper (NeuralFluid,
arXiv 2405.14903):

* ``mac``        -- MAC grid, the gradient matrix G (Sec. Numerical Simulation)
* ``geometry``   -- signed distances, face fluid fractions alpha by marching
                    squares (Sec. Projection, cut-cell paragraph), solid velocity
* ``advection``  -- RK2 semi-Lagrangian advection (Eq. advection_matrix;
                    App. B Eqs. advection_1 / advection_2)
* ``projection`` -- variational pressure projection (Eqs. projection_matrix,
                    u_next_matrix) and a converged FP64 solve
* ``step``       -- one full step, its tangent (JVP) and adjoint (VJP)
                    (Sec. Back-propagation through Time / through Geometry)
* ``rollout``    -- rigid ellipsoid pose dynamics, losses, BPTT

Parity status of each function is stated in its module header.
"""
