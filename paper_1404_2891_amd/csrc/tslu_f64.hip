// Tournament local LUs, FP64 storage.
#include "tslu_local.h"

namespace fm {
template int tslu_local_launch<double>(dim3, const LUDev*, int, int, int, int, int, hipStream_t);
}  // namespace fm
