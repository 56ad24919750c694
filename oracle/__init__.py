"""FP64 CPU oracle (test infrastructure only; the GPU library never imports it)."""
