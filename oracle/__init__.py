"""FP64 CPU oracle of the fluctuating LB method (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the HIP path.
"""
