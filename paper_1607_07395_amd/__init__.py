"""CABS on AMD MI355X: cascaded bilateral sampling (arXiv:1607.07395) in HIP for gfx950.

The compute path is the C-ABI library ``libcabs.so`` (include/cabs.h); the
submodule ``api`` only marshals arguments to it (``from paper_1607_07395_amd
import api``), ``build`` compiles it.
"""
