// Single-domain kernels instantiated for the D3Q39 lattice.
#include "ops_impl.hpp"

ESBGK_INSTANTIATE_LATTICE(esbgk::LatD3Q39, d3q39)
