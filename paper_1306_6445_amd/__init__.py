"""MI355X-native D2Q9 pseudopotential MRT lattice Boltzmann step with the
surface-tension source term (Li & Luo, arXiv:1306.6445).

The compute path is the HIP library ``liblbm_mi355x.so`` behind the C ABI in
``include/lbm.h``; ``paper_1306_6445_amd.lbm`` is its ctypes binding and
``paper_1306_6445_amd.workloads`` builds seeded synthetic inputs.
"""
