"""MI355X-native face-graph finite-volume PISO library (DiFVM hot path).

The compute path lives in the HIP/C++ shared library ``libdifvm.so`` (``csrc/``), reached through the
C-ABI declared in ``include/difvm.h``.  ``binding`` marshals arguments to it with ctypes; ``meshgen``
builds seeded synthetic inputs.  Importing this package loads nothing native: the library is loaded
by ``binding.lib()`` on first use, and raises if it has not been built.
"""
__all__ = ["binding", "meshgen"]
