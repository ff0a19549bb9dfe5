// Tile-pass kernels: double, forward.
#define TQS_T double
#define TQS_BWD false
#define TQS_LAUNCH_NAME launch_pass_f64_fwd
#define TQS_ATTR_NAME pass_attrs_f64_fwd
#include "pass_tu.inc"
