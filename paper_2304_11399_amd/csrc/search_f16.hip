// Search kernels of libens for f16 trace storage (see search.h).
#include "search.h"

namespace ens {
template hipError_t launch_search_dt<DT_F16>(int, int, int, int, const SearchArgs &, int32_t, hipStream_t);
}  // namespace ens
