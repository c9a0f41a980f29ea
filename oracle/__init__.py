"""Plain FP64 CPU oracle for the FETI dual operator (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library; both read their
inputs from the seeded problem generator in ``synth``.
"""
