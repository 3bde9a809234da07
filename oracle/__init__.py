"""FP64 CPU oracle of the NTU bond update (test infrastructure only)."""
