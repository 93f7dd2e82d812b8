"""FP64 CPU oracle of the simple-update hot path (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  It shares no code with the GPU library.
"""
