// sbr_backward.hip -- adjoint of the SBR radio map (placeholder until the
// reverse sweep lands).
#include "rt_internal.h"

rt_status rt_launch_backward(const BwdLaunch&, hipStream_t) {
    return rt_fail(RT_EUNSUPPORTED, "rt_radio_map_backward: not built yet");
}
