"""MI355X-native central-moment lattice Boltzmann stream-and-collide.

The compute path is the HIP library ``liblbm.so`` (C ABI declared in
``include/lbm.h``); ``paper_2203_01316_amd.lbm`` is its thin ctypes binding and
``paper_2203_01316_amd.workloads`` builds seeded synthetic inputs.
"""

__all__ = ["lbm", "workloads"]
