"""MI355X (gfx950) implementation of the explicit-implicit domain-splitting
hot path of May & Thein (arXiv 2211.00705): explicit HLL sweep over bulk
cells, dual time stepping on the implicit zones around tiny cut cells, and
the two-phase interface Riemann solve, behind the C ABI of include/imexds.h.

``paper_2211_00705_amd.imexds`` is the ctypes binding; importing it loads
libimexds.so and fails loudly if the library is missing.
"""
__all__ = ["imexds", "workloads", "build"]
