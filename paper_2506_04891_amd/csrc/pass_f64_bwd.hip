// Tile-pass kernels: double, backward.
#define TQS_T double
#define TQS_BWD true
#define TQS_LAUNCH_NAME launch_pass_f64_bwd
#define TQS_ATTR_NAME pass_attrs_f64_bwd
#include "pass_tu.inc"
