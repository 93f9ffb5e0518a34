"""CPU FP64 oracle (test infrastructure only; see pw_oracle)."""
