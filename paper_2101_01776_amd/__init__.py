"""MI355X-native solver of the nonlinear stage equations of fully implicit
Runge-Kutta methods (Gauss, Radau IIA) for method-of-lines PDEs.

The compute path is the HIP library ``libirk.so`` (C ABI in include/irk.h);
``paper_2101_01776_amd.irk`` is its ctypes binding, ``inputs`` the seeded
synthetic workloads.  Importing the package does not load the library; the
first call into ``irk`` does, and raises if it has not been built.
"""
__all__ = ["irk", "inputs"]
