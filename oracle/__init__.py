"""CPU oracle (test infrastructure only; see qilbm_oracle)."""
