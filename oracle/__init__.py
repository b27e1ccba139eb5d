"""GridShift FP64 CPU oracle: test infrastructure only (see gs_oracle.c)."""
