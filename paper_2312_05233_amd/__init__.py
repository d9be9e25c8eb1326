"""TNEP (arXiv:2312.05233) dipole / polarizability evaluation and spectra on
AMD Instinct MI355X (gfx950): HIP kernels behind the C ABI in include/tnep.h.

The binding lives in ``paper_2312_05233_amd.tnep`` (loaded on first use);
``paper_2312_05233_amd.build`` compiles libtnep.so in-tree.
"""

__all__ = ["tnep", "build"]
