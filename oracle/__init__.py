"""FP64 CPU oracle -- test infrastructure only.

Imported by the test suite, the smoke check and the benchmark's CPU-baseline leg; never by
the library. See ``bm_oracle`` for what it computes and the readings it takes.
"""
