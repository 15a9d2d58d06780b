"""MI355X-native finite element numerical integration for first-order
approximations (element stiffness matrices and load vectors of affine
tetrahedra and 6-node prisms; scalar convection-diffusion-reaction and
3-component elasticity), after Banas, Kruzel and Bielanski, arXiv:1504.01023.

The compute path is the C-ABI library ``libfe.so`` (hand-written HIP for
gfx950); :mod:`paper_1504_01023_amd.fe` is its thin Python binding. Importing
this package loads nothing; the binding loads the library on first use and
raises if it is missing.
"""
__all__ = ["fe", "inputs"]
