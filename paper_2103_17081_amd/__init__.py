"""MI355X-native inexact-subdomain Schwarz solver for the 2D Dirichlet Helmholtz problem.

The package is deliberately thin: the solver lives in the HIP/C++ shared library
``libddhelm.so`` (built from ``csrc/``), and ``binding`` only marshals arguments to
its C ABI.  ``inputs`` holds the seeded synthetic input generators.  Nothing is
imported eagerly, so importing the package never touches the GPU.
"""

__all__ = ["inputs", "binding"]
