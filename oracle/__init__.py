"""FP64 CPU oracle of the DAETI monodomain method (test infrastructure only)."""
