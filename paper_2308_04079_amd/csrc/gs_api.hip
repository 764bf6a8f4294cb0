// The one synchronising call of the C ABI: reading the device status word.
#include "gs_internal.h"

using namespace gs;

extern "C" int gs_read_status(const gs_instances* inst, uint32_t* status, uint32_t* count,
                              gs_stream_t stream) {
  if (!inst || !inst->status || !inst->count) return GS_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return GS_ERR_HIP;
  uint32_t st = 0, ct = 0;
  if (hipMemcpy(&st, inst->status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return GS_ERR_HIP;
  if (hipMemcpy(&ct, inst->count, sizeof(ct), hipMemcpyDeviceToHost) != hipSuccess) return GS_ERR_HIP;
  if (status) *status = st;
  if (count) *count = ct;
  if (st & GS_STATUS_CAPACITY) return GS_ERR_CAPACITY;
  if (st & GS_STATUS_SORT) return GS_ERR_SORT;
  return GS_OK;
}
