"""MI355X-native checkerboard spin-glass Monte Carlo (Metropolis / heat bath,
Parisi-Rapuano random numbers).

The compute path is the C-ABI library ``libsg.so`` built from ``csrc/``;
``binding`` marshals arguments to it.  Importing this package does not load
the library; ``binding.lib()`` does, and raises if it is missing.
"""
SG_CONVENTIONS_VERSION = 1
