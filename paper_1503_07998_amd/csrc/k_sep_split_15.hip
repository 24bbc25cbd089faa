// Split-view backward pass with 16-row groups, 15-tap bucket.
#define MVD_SEP_G 16
#define MVD_SEP_NS sepk16
#include "k_sep_impl.hpp"
MVD_SEP_INSTANTIATE_SPLIT(15)
