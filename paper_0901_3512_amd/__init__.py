"""Seed-CG on AMD MI355X (gfx950): HIP kernels behind a C ABI, with a thin Python binding.

Build with paper_0901_3512_amd.build.build(); the binding refuses to run without the
compiled library.
"""
from .seedcg import SeedCG, SeedCGBatch, SeedCGError, load_library, LIB_PATH, exported_symbols, probe_bandwidth, probe_mfma

__all__ = ["SeedCG", "SeedCGBatch", "SeedCGError", "load_library", "LIB_PATH", "exported_symbols", "probe_bandwidth",
           "probe_mfma"]
