// Kernel instantiations for the FFT lengths of one family (TBS_LENGTHS_FIVE).
#include "tbs_passes.hpp"

namespace tbs {
TBS_FAMILY_DISPATCH(dispatch_five, TBS_LENGTHS_FIVE)
}  // namespace tbs
