"""MI355X (gfx950) preconditioned GCR(k) solver for the elliptic depth problem of
a semi-implicit shallow-water model on a lon/lat grid (arXiv:2103.16120).

Import ``paper_2103_16120_amd.lib`` for the binding of the HIP library; it
raises if the library has not been built.  Building: ``python -m
paper_2103_16120_amd.build``.
"""
__all__ = ["lib", "build"]
