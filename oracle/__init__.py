"""FP64 CPU oracle of the strong-field QED step (test infrastructure only)."""
