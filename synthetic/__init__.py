"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package stands in for the paper's DFT ground states of real molecules
(experimental geometries, pseudopotentials and an external DFT code, none of
which exist here).  It draws a molecule-in-a-box local potential made of
Gaussian wells, random perturbing potentials and frequency lists, and it
produces the lowest eigenpairs of the model Hamiltonian that play the role of
the DFT valence states.  It holds none of the polarizability, Sternheimer or
Lanczos arithmetic: those live, independently, in the oracle and in the HIP
library.
"""
from .workloads import (CONFIGS, Workload, make_workload, gaussian_wells,
                        random_potentials, smooth_directions, imag_freqs, real_freqs, HA_PER_EV)
from .ground_state import ground_state

__all__ = ["CONFIGS", "Workload", "make_workload", "gaussian_wells",
           "random_potentials", "smooth_directions", "imag_freqs", "real_freqs", "ground_state",
           "HA_PER_EV"]
