"""FP64 CPU oracle of the MDF-LBM hot path (test infrastructure only)."""
