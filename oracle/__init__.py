"""FP64 CPU oracle (test infrastructure only; see lbm_oracle.cpp)."""
