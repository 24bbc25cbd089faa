// Separable forward pass kernels for kernel sizes up to 41 (the bucket's
// backward and single-input passes: k_sep_41_bwd.hip, k_sep_41_single.hip).
#include "k_sep_impl.hpp"
#include "k_sep_units.hpp"

MVD_SEP_INSTANTIATE_FWD(41)
