"""FP64 CPU oracle for the Parareal method for the Cahn-Hilliard equation.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously-correct
definition that the HIP path is checked against.  Only the test suite, the
``smoke()`` check and the benchmark's CPU-baseline leg may import it; the
product library never does, and it shares no code, tables or constants with it.

Everything is float64 NumPy/SciPy, written from the paper:
  * ``operators``   -- the Dirichlet difference Laplacian D_h (Section 3) and
                       its 2D extension (Section 3, Remark item 2).
  * ``schemes``     -- the time steps (2.3) (Eyre, solved by the Newton form
                       of Section 3, NPA-II), (2.4) and (2.5), plus the fully
                       implicit backward-Euler variant.
  * ``propagators`` -- F (J fine steps of dt = dT/J) and G (coarse steps).
  * ``parareal``    -- the predictor-corrector iteration (2.2).
  * ``energy``      -- the discrete Ginzburg-Landau energy of (1.2).
  * ``linear_model``-- the linearised propagators P_i, P_{J_i} of Section 3
                       and the convergence bound of Theorems 3.7/3.9/3.11.
  * ``dd``          -- the Neumann-Neumann domain-decomposition solve of the
                       PA-I fine step (2.4) in 1D (Section 4).
  * ``nn``          -- FP64 reference forward/backward of the convolutional
                       surrogate used as a learned coarse propagator.
Each function cites the passage it follows.
"""
