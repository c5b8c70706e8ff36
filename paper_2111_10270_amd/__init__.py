"""MI355X-native BDD Lagrange-decomposition solver for 0-1 ILPs.

The solver itself lives in the HIP/C++ shared library built from ``csrc/``;
``binding`` marshals arguments to its C ABI.  Nothing is imported eagerly so
that the instance generators can be used without loading the library.
"""
