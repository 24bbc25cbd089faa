// Instantiation units of the separable passes for the largest kernel-size
// buckets: the forward, backward and single-input dispatchers of one bucket in
// translation units of their own, each in its own namespace (MVD_SEP_NS), so
// that they compile in parallel.  Included after k_sep_impl.hpp.
#pragma once

#define MVD_SEP_INSTANTIATE_FWD(KB)                                                        \
  namespace mvd {                                                                          \
  hipError_t sep_forward_kb##KB(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {  \
    return MVD_SEP_NS::forward_bucket<KB>(a, p, s);                                        \
  }                                                                                        \
  }

#define MVD_SEP_INSTANTIATE_BWD(KB)                                                        \
  namespace mvd {                                                                          \
  hipError_t sep_backward_kb##KB(const SepPassArgs &a, const SepPlan &p, hipStream_t s) { \
    return MVD_SEP_NS::backward_bucket<KB>(a, p, s);                                       \
  }                                                                                        \
  }

#define MVD_SEP_INSTANTIATE_SINGLE(KB)                                                     \
  namespace mvd {                                                                          \
  hipError_t sep_single_kb##KB(const SepPassArgs &a, const SepPlan &p, int ep, hipStream_t s) { \
    return MVD_SEP_NS::single_bucket<KB>(a, p, ep, s);                                     \
  }                                                                                        \
  }
