// Search kernels of libens for f32 trace storage (see search.h).
#include "search.h"

namespace ens {
template hipError_t launch_search_dt<DT_F32>(int, int, int, int, const SearchArgs &, int32_t, hipStream_t);
}  // namespace ens
