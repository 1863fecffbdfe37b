"""FP64 CPU oracle for the coupled LLG + cavity-mode stepper.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library and its Python
binding never do, and it imports nothing from them.

Modules:
  newell   - cell-averaged demag tensor (closed form + far-field quadrature),
             FFT and direct-sum demag fields
  model    - effective field, LL torque, mode-weighted average, cavity RHS
  stepper  - RK4 and Dormand-Prince 5(4) joint stepping, controller, trace
  theory   - closed forms of the coupled-mode theory used as pins
  spectrum - spectra and peak picking of sampled traces

Parity pins for each part are in tests/test_oracle_*.py.
"""
