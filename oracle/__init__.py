"""FP64 CPU oracle (test infrastructure only; see tdb_oracle)."""
