"""MI355X (gfx950) FP64 hydro step: PPM reconstruction at 26 quadrature points,
central-upwind Kurganov-Tadmor flux with Simpson face quadrature, and the
finite-volume divergence, on batches of 8^3 subgrids with 3 ghost layers.

Modules: ``hydro`` (binding of the C ABI in include/hydro.h), ``inputs``
(seeded synthetic workloads), ``serving`` (continuous-batching request loop),
``build`` (hipcc build of libhydro.so).
"""
