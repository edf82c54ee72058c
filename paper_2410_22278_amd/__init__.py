"""MI355X-native Gamma-point periodic J/K build with Ewald splitting.

Importing the package does not load the HIP library; `paper_2410_22278_amd.pbcjk`
does (and fails loudly when the built library is missing).
"""
__all__ = ["inputs"]
