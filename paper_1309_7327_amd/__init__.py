"""MI355X-native right-hand side of the reacting compressible Navier-Stokes
equations (eighth-order centred and narrow stencils, thermochemistry) and its
multirate spectral-deferred-correction step, behind the C-ABI library
libnarrowsdc.so (see include/narrowsdc.h)."""
