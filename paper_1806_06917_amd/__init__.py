"""MI355X (gfx950) peridynamics hot path: neighbour lists, bond-force gather
with critical-stretch damage, velocity-Verlet stepping and the matrix-free
tangent inside CG, after Diehl et al., arXiv:1806.06917.

``paper_1806_06917_amd.pd`` binds the HIP library (libpd_hip.so);
``paper_1806_06917_amd.inputs`` generates seeded synthetic workloads.
"""
