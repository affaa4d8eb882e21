"""MI355X (gfx950) Barnes-Hut treecode for single-particle Metropolis Monte
Carlo of charged systems, after Gan & Xu's octree method with local tree
adjustment.  The compute path is the HIP library libbhmc.so (C ABI in
include/bhmc.h); ``paper_1305_1825_amd.bhmc`` is its Python binding and
``paper_1305_1825_amd.workloads`` draws seeded synthetic systems."""
