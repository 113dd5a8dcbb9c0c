// Batched kernels instantiated for the D3Q39 lattice.
#include "batch_impl.hpp"

ESBGK_INSTANTIATE_BATCH(esbgk::LatD3Q39, d3q39)
