// Single-domain kernels instantiated for the D2Q33 lattice.
#include "ops_impl.hpp"

ESBGK_INSTANTIATE_LATTICE(esbgk::LatD2Q33, d2q33)
