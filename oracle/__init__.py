"""CPU FP64 oracle of the relativistic lattice Boltzmann step (test infrastructure only)."""
