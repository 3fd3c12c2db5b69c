"""MI355X-native fractional-step MRT lattice Boltzmann for two-phase flow.

The compute path lives in the HIP library ``liblbm2p.so`` (sources under
``csrc/``, C declarations in ``include/lbm2p.h``); ``binding`` marshals
arguments to it through ctypes.  ``inputs`` builds seeded initial fields.
The binding is imported lazily so that ``inputs`` can be used without a GPU.
"""
