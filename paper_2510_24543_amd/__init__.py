"""MI355X-native preconditioned nonlinear CG ground-state solver for two-component
dipolar Bose-Einstein condensates with LHY corrections (arXiv:2510.24543).

The compute path is the HIP library behind include/bec.h; import
``paper_2510_24543_amd.solver`` for the torch-facing API (it loads the library
and fails loudly when it has not been built).  ``paper_2510_24543_amd.inputs``
holds the seeded synthetic workloads and imports nothing else from here.
"""
