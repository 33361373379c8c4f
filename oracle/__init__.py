"""FP64 CPU oracle of the PAM hot path (test infrastructure only)."""
