"""MI355X-native ternary free-energy lattice Boltzmann + immersed-boundary
library (Pepona et al., "Modelling ternary fluids in contact with elastic
membranes").

The compute path lives in the HIP shared library ``liblbib.so`` built from
``csrc/``; :mod:`paper_1906_03065_amd.lbib` is its ctypes binding and
:mod:`paper_1906_03065_amd.workloads` holds the seeded synthetic inputs.
Importing this package loads nothing; the binding loads the library on first
use and raises if it has not been built.
"""
__all__ = ["lbib", "workloads"]
