// Single-domain kernels instantiated for the D2Q37 lattice.
#include "ops_impl.hpp"

ESBGK_INSTANTIATE_LATTICE(esbgk::LatD2Q37, d2q37)
