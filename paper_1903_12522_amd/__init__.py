"""MI355X-native controllability-method (CMCG) solver for the Helmholtz equation.

The solver is the HIP library ``libcmcg.so`` (sources in ``csrc/``, C ABI in
``include/cmcg.h``); ``paper_1903_12522_amd.cmcg`` is its Python binding and
``paper_1903_12522_amd.serving`` the continuous-batching request loop.  Importing the package
itself loads nothing; importing the binding fails loudly if the library is not built.
"""

__all__ = ["cmcg", "build"]
