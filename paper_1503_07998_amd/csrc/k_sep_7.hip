// Separable pass kernels for kernel sizes up to 7 (one bucket per file).
#include "k_sep_impl.hpp"

MVD_SEP_INSTANTIATE(7)
