"""CPU oracle for the STZ hot path (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never uses it.
"""
