// Kernel instantiations for the FFT lengths of one family (TBS_LENGTHS_POW2).
#include "tbs_passes.hpp"

namespace tbs {
TBS_FAMILY_DISPATCH(dispatch_pow2, TBS_LENGTHS_POW2)
}  // namespace tbs
