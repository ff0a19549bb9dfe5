// Tile-pass kernels: float, backward.
#define TQS_T float
#define TQS_BWD true
#define TQS_LAUNCH_NAME launch_pass_f32_bwd
#define TQS_ATTR_NAME pass_attrs_f32_bwd
#include "pass_tu.inc"
