"""FP64 CPU oracle (test infrastructure only; the GPU path never imports it)."""
