// vc_pending.hip -- entry points whose kernels are not built yet; they validate nothing and
// report VC_ERROR_UNSUPPORTED_CODEC so that callers fail loudly.
#include "vc_internal.hpp"

extern "C" {

vc_status vc_batch_plan_create(vc_batch_plan** plan, const vc_codec*, const vc_segment*, int, hipStream_t)
{
  if (plan) *plan = nullptr;
  return VC_ERROR_UNSUPPORTED_CODEC;
}
vc_status vc_batch_plan_run(vc_batch_plan*, hipStream_t) { return VC_ERROR_UNSUPPORTED_CODEC; }
vc_status vc_batch_plan_run_separate(vc_batch_plan*, hipStream_t) { return VC_ERROR_UNSUPPORTED_CODEC; }
vc_status vc_batch_plan_destroy(vc_batch_plan*) { return VC_SUCCESS; }

}
