"""FP64 CPU oracle for the peridynamic hot path (test infrastructure only)."""
