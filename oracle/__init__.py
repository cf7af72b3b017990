"""FP64 CPU oracle of the PINN residual loss and gradient (test infrastructure only)."""
