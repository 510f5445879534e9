// Instantiates every pass kernel for one transform length (HG_LEN, set by the
// build) and exposes them through a kernel table; one object per length lets
// the lengths compile in parallel.
#include "kernels.hpp"

#ifndef HG_LEN
#error "HG_LEN must be defined"
#endif

#define HG_CAT2(a, b) a##b
#define HG_CAT(a, b) HG_CAT2(a, b)

namespace hg {
const LengthEntry* HG_CAT(length_entry_, HG_LEN)() {
  static const LengthEntry e = make_length_entry<HG_LEN>();
  return &e;
}
}  // namespace hg
