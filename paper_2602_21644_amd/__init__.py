"""MI355X-native (gfx950) MP-weighted Gaussian-splatting hot path.

The compute lives in a HIP/C-ABI shared library (libgs.so, declared in
include/gs.h); this package is its thin Python binding (`gs`), a torch
autograd wrapper, tracking/mapping loops and the seeded synthetic input
generator (`synth`). Importing the package loads nothing; `gs.lib()` loads
the library and raises if it has not been built.
"""
