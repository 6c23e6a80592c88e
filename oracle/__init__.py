"""FP64 CPU oracle for the GDM hot path.  Test infrastructure only: imported by
the test-suite, the smoke check and the benchmark's CPU-baseline leg, never by
the product library or its binding."""
