"""FP64 CPU oracle of the HDP hot path (test infrastructure only)."""
