// Kernel instantiations for the FFT lengths of one family (TBS_LENGTHS_THREE).
#include "tbs_passes.hpp"

namespace tbs {
TBS_FAMILY_DISPATCH(dispatch_three, TBS_LENGTHS_THREE)
}  // namespace tbs
