"""MI355X (gfx950) implementation of MPO-times-MPS apply + variational compression
(SeeMPS, arXiv 2601.16734): a C-ABI HIP library and its thin Python binding.

Importing the package loads nothing; `binding.load()` opens the built library
and fails loudly when it is missing.
"""

__all__ = ["binding", "build"]
