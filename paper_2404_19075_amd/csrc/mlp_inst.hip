// mlp_inst.hip -- explicit instances of the fused MLP kernel for one precision
// and mode (DINR_INST_PREC, DINR_INST_MODE), both supported shapes and both
// hidden activations (Swish only in the group mode).  The build compiles this file once per (precision,
// mode) so that the instances compile in parallel.
#include "mlp.h"

#if !defined(DINR_INST_PREC) || !defined(DINR_INST_MODE)
#error "compile with -DDINR_INST_PREC=<0|1> -DDINR_INST_MODE=<0..4>"
#endif
// the group mode (4) exists for Swish networks only
#define MODE_GROUP_VALUE 4

namespace dinr {

static_assert(MODE_GROUP == MODE_GROUP_VALUE, "group mode number");

#define DINR_INST(IN, H, ACT)                                                          \
  template hipError_t mlp_launch<DINR_INST_PREC, IN, H, DINR_INST_MODE, ACT>(          \
      const MlpArgs&, int, hipStream_t);
#if DINR_INST_MODE != MODE_GROUP_VALUE
DINR_INST(128, 64, 0)
DINR_INST(256, 256, 0)
#endif
DINR_INST(128, 64, 1)
DINR_INST(256, 256, 1)
#undef DINR_INST

}  // namespace dinr
