"""Sparse-geometry lattice Boltzmann on MI355X (gfx950).

A uniform mesh of fixed-size tiles covers the geometry; only tiles holding at
least one non-solid node are stored, and PDFs cross tile edges through a
tile-neighbour map (Tomczak & Szafran, arXiv 1703.08015, Sec. 3).  The time
step -- BGK quasi-compressible collision fused with gather streaming and
half-way bounce-back -- runs in hand-written HIP kernels behind the C ABI
declared in ``include/lbm.h``; ``paper_1703_08015_amd.lbm`` is the thin Python
binding (argument marshalling only) and ``inputs`` draws seeded geometries.
"""
