// One (precision, spreading mode) instantiation of the batched kernel; the
// build compiles this file once per pair (OT_INST_T, OT_INST_MODE).
#include "batch_kernels.h"

#ifndef OT_INST_T
#error "OT_INST_T and OT_INST_MODE select the instantiation"
#endif

namespace ot {
template int enqueue<OT_INST_T, OT_INST_MODE>(ot_batch_plan *p, const void *field, const void *force, const void *pos,
                                             int32_t *ids, void *vel, void *fout, void *grad, hipStream_t s);
template const void *kbatch_fn<OT_INST_T, OT_INST_MODE>(bool grad, bool small);
template const void *hm_fn<OT_INST_T, OT_INST_MODE>(int ops);
}  // namespace ot
