// sbr_batched.hip -- batched transmitters / material samples (placeholder).
#include "rt_internal.h"

rt_status rt_launch_batched(const BatchLaunch&, hipStream_t) {
    return rt_fail(RT_EUNSUPPORTED, "rt_radio_map_batched: not built yet");
}
