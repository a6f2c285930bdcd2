// Tournament local LUs, FP32 storage.
#include "tslu_local.h"

namespace fm {
template int tslu_local_launch<float>(dim3, const LUDev*, int, int, int, int, int, hipStream_t);
}  // namespace fm
