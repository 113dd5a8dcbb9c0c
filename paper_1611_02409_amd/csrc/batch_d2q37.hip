// Batched kernels instantiated for the D2Q37 lattice.
#include "batch_impl.hpp"

ESBGK_INSTANTIATE_BATCH(esbgk::LatD2Q37, d2q37)
