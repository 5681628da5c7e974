"""MI355X-native coupled phase-field lattice Boltzmann step for two-phase EHD."""
