"""FP64 CPU oracle (test infrastructure only; see gmrf_oracle.py)."""
