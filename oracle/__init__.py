"""FP64 CPU oracle for the subset-DIC hot path (test infrastructure only)."""
