"""MI355X (gfx950) solver for the even-parity anisotropic RTE: the preconditioned Richardson
iteration of Doelz, Palii and Schlottbom (arXiv:2102.09038) behind the C ABI of
``include/rte.h``.

Submodules: ``inputs`` (seeded synthetic instances), ``rte`` (ctypes binding of librte,
imported lazily because it loads the HIP library), ``build`` (hipcc build of librte.so).
"""
__all__ = ["inputs", "build"]
