// Separable backward pass kernels for kernel sizes up to 41.
#define MVD_SEP_NS sepkb
#include "k_sep_impl.hpp"
#include "k_sep_units.hpp"

MVD_SEP_INSTANTIATE_BWD(41)
