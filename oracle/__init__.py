"""FP64 CPU oracle of the hybrid marcher (test infrastructure only)."""
