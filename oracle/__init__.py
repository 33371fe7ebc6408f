"""FP64 CPU oracle of the tracker (test infrastructure only; see ccpt_oracle)."""
