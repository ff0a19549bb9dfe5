// Tile-pass kernels: float, forward.
#define TQS_T float
#define TQS_BWD false
#define TQS_LAUNCH_NAME launch_pass_f32_fwd
#define TQS_ATTR_NAME pass_attrs_f32_fwd
#include "pass_tu.inc"
