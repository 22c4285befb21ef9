// One (precision, spreading mode) instantiation of the plain-launch kernels;
// the build compiles this file once per pair (OT_INST_T, OT_INST_MODE).
#include "track_kernels.h"

#ifndef OT_INST_T
#error "OT_INST_T and OT_INST_MODE select the instantiation"
#endif

namespace ot {
template int dispatch_ops<OT_INST_T, OT_INST_MODE>(int ops, const ot_tree *t, dim3 g, dim3 b, int64_t tile,
                                                   hipStream_t s, int64_t n, const void *pos, const void *field,
                                                   const void *force, int32_t *ids, void *vel, void *fout, void *grad,
                                                   const FxWs &ws, const int32_t *hid);
}  // namespace ot
