"""MI355X-native CTD solver for the Allen-Cahn equation (arXiv 2410.15519).

The compute path is the HIP library libctd.so (built in-tree for gfx950);
`paper_2410_15519_amd.ctd` is its ctypes binding.  Importing the binding
raises ImportError when the library is missing -- there is no CPU fallback.
"""
__all__ = ["ctd"]
