"""MI355X-native integral-direct J/K build (Rys-quadrature ERIs digested with D).

The compute path is the C-ABI library built from ``csrc/`` (HIP for gfx950); the
Python module ``jk`` only marshals arguments to it.
"""
