"""MI355X-native EBIT interface step (Pan et al., arXiv 2309.00338).

`paper_2309_00338_amd.ebit` binds the gfx950 library (libebit.so); the input
generators live in `paper_2309_00338_amd.inputs`. Importing the package does
not load the library, so the generators stay usable on hosts without it.
"""
