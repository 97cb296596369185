"""CPU oracle of the RSRR method: TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with it.
"""
