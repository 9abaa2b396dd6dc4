"""FP64 CPU oracle for the batched DC-loadflow screen (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the solver library never imports it.
"""
