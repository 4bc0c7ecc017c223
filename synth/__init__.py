"""Seeded synthetic inputs for the Seed-CG solver and its oracle.

This package draws the random gauge links, smears them, and builds the sources.
It holds none of the solver's arithmetic (no Dirac operator, no Krylov method):
both the HIP library's tests and the oracle read the same arrays from here.

Canonical layouts (shared with the C ABI):
  * site index  s = x + Lx*(y + Ly*(z + Lz*t)),  parity (x+y+z+t) mod 2;
  * links       complex128 array (4, V, 3, 3): U_mu(s)[a, b], mu = x, y, z, t,
                the link from s to s + mu-hat, with no boundary sign folded in;
  * spinors     complex128 array (n, Vh, 4, 3) on the even sites, listed in
                increasing s; component (spin, colour).
"""
from .links import random_su3_links, ape_smear, plaquette
from .sources import point_sources, gaussian_sources, z2_sources
from .configs import CONFIGS, SolverConfig, make_inputs, kappa_for

__all__ = [
    "random_su3_links", "ape_smear", "plaquette",
    "point_sources", "gaussian_sources", "z2_sources",
    "CONFIGS", "SolverConfig", "make_inputs", "kappa_for",
]
