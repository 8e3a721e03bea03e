"""FP64 CPU oracle of the strength-SPH hot path (test infrastructure only)."""
