// Batched kernels instantiated for the D2Q33 lattice.
#include "batch_impl.hpp"

ESBGK_INSTANTIATE_BATCH(esbgk::LatD2Q33, d2q33)
