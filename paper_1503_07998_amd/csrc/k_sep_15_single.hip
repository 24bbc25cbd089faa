// Single-input separable passes (the reverse sweep's and the low-rank terms'
// epilogues) for kernel sizes up to 15.
#define MVD_SEP_NS sepks
#include "k_sep_impl.hpp"
#include "k_sep_units.hpp"

MVD_SEP_INSTANTIATE_SINGLE(15)
