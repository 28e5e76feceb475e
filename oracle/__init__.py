"""FP64 CPU oracle for the NLINV hot path.  Test infrastructure only: imported
by the test suite, the smoke check and the benchmark's CPU-baseline leg."""
