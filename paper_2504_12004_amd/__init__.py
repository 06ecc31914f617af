"""MI355X-native Scaled Block Vecchia (SBV) log-likelihood.

The compute path is the HIP/C-ABI library libsbv.so (csrc/); this package only
marshals arguments to it.  Importing the package does not load the library;
the first call does, and it fails loudly if the library is missing.
"""
__all__ = ["sbv", "synth"]
