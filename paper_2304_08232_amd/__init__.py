"""MI355X-native multigrid-preconditioned CG for the 27-point HPCG stencil.

The solver is the HIP library libmgpcg.so (C ABI: include/mgpcg.h); this
package holds its sources (csrc/), its build step (build.py), the Python
binding (mgpcg.py) and the seeded synthetic input generators (inputs.py).
"""
