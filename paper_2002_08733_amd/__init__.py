"""MI355X-native matrix-free DG time-domain Maxwell solver (libmdg binding).

Importing this package does not load the native library; ``Solver`` does, and
fails loudly if ``libmdg.so`` has not been built (``python -m
paper_2002_08733_amd.build``).
"""
from .mdg import MdgError, Solver, load_library  # noqa: F401
