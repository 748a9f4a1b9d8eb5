"""CPU oracle for the Wirtinger-Jacobian gain-calibration hot path.

TEST INFRASTRUCTURE ONLY.  Plain, slow, complex128 NumPy written from Smirnov &
Tasse, "Radio interferometric gain calibration as a complex optimization
problem" (MNRAS 2015).  Only the tests, the smoke entry point and the CPU
baseline leg of the benchmark may import it; the GPU library never does, and
it shares no code with the GPU library (inputs come from the seeded generators
in ``paper_1502_06974_amd.synth``, which contain none of the method).

Modules
  calib     -- the algorithm layer: per-antenna J^H J / J^H D accumulation,
               StefCal (scalar and 2x2), CohJones, AllJones, residuals, the
               GN / lambda=1 average schedule and the convergence test.
  jacobian  -- the definition layer: explicit complex Jacobians from the
               Wirtinger derivatives of the measurement equation, full
               complex Gauss-Newton and Levenberg-Marquardt on tiny arrays,
               and the 4x4 forms of the 2x2 matrix operators.
  mlp       -- float64 forward/backward of the warm-start network.
"""
